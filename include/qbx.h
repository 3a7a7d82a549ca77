/*
 * qbx.h -- C ABI of libqbx, the MI355X (gfx950) hot path of Quadrature by
 * Expansion (QBX) for the 2D Helmholtz single-layer (S) and double-layer (D)
 * potentials (Kloeckner, Barnett, Greengard, O'Neil, "Quadrature by
 * Expansion: A New Method for the Evaluation of Layer Potentials").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers unless marked "host".  Complex
 *    values are interleaved (re, im) doubles, the layout of torch.complex128.
 *  - The caller owns every buffer.  The library never allocates, never frees
 *    and keeps no pointer after a call returns; scratch memory comes from the
 *    caller's workspace `ws` of `ws_bytes` bytes (sizes from the *_bytes
 *    queries below, alignment 256 bytes).
 *  - Work is enqueued on `stream` and is stream-ordered; no call synchronizes
 *    the device except the ones documented as synchronous.  Calls that use
 *    different workspaces may run concurrently.
 *  - Return value: 0 on success, a negative qbx_status otherwise.  Argument
 *    validation happens on the host before anything is enqueued, so invalid
 *    arguments never reach the GPU.  qbx_strerror() names a code;
 *    qbx_last_error() gives the message of the last failure on this thread.
 *
 * Geometry (Section 4.1 of the paper): a closed counter-clockwise curve split
 * into n_panels panels, each carrying q = 16 nodes placed at the 16-point
 * Gauss-Legendre abscissae of the panel parameter (ascending); the panel is
 * the degree-15 polynomial through its nodes.  nodes[n_panels][16][2].
 * Targets are the nodes themselves (the Nystrom grid, Section 3.4.2), in node
 * order; T = 16*n_panels.
 *
 * Source grid (Section 3.4.2, Section 4.1): on every panel, the
 * q_s = 16*oversample point Gauss-Legendre rule of the same panel; the
 * density is interpolated there from its node values.
 *
 * Centers (Section 3.3, step 4(a)): c = x + s*r*h_m*n at every target x of
 * panel m, s = +1 exterior, -1 interior; n the outward unit normal; h_m the
 * panel arc length by the source rule; radius R = r*h_m (the paper takes
 * r = 1/2).
 *
 * Output: the one-sided limits (Section 3.3, step 4(c))
 *   u(x) = (i/4) sum_{l=-p..p} a_l J_l(k R) e^{i l theta},  theta = arg(x - c),
 *   a_l  = sum_j w_j sigma_j H^(1)_l(k|x'_j - c|) e^{-i l theta'_j}      (S),
 * and for D the same with d/dn' of the source factor applied to mu
 * (Section 2 eq. graf-coefficient, Section 3.2 eq. graf-coefficient-dlp; the
 * paper's e^{+il theta'} / e^{-il theta} convention is the same sum under
 * l -> -l).  The principal value of D is the average of both limits
 * (Section 3.2, eq. dlp-twosided).
 * Layout out[n_sides][n_kinds][T] complex: for side = QBX_BOTH the exterior
 * limit comes first; kinds in the order S, D.
 */
#ifndef QBX_H
#define QBX_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QBX_Q 16             /* nodes per panel (Section 4.1)                  */
#define QBX_PMAX 24          /* largest supported expansion order p            */
#define QBX_OVERSAMPLE_MAX 8 /* source nodes per panel = 16*oversample <= 128  */

enum qbx_kind { QBX_S = 1, QBX_D = 2 };                       /* bit mask; S|D fused */
enum qbx_side { QBX_INTERIOR = -1, QBX_BOTH = 0, QBX_EXTERIOR = 1 };

enum qbx_status {
  QBX_OK = 0,
  QBX_EINVAL = -1,     /* null pointer, n_panels < 3, q != 16, p < 0 or p > QBX_PMAX,
                          k <= 0 or not finite, r <= 0 or not finite, oversample < 1
                          or > QBX_OVERSAMPLE_MAX, bad side or kind, bad item        */
  QBX_EWORKSPACE = -2, /* ws_bytes smaller than the matching *_bytes query           */
  QBX_EORIENT = -3,    /* clockwise contour (negative signed area)                   */
  QBX_EGRAF = -4,      /* a source lies inside a center's disk: Graf's condition
                          |x - c| < |x' - c| (Section 2, eq. x-c-closest) fails     */
  QBX_EDEVICE = -5,    /* a HIP call failed; see qbx_last_error()                  */
  QBX_EIO = -6         /* an autotuner cache file could not be read or written, or
                          holds a malformed entry                                    */
};

typedef struct {
  int32_t n_panels;     /* >= 3                                                  */
  int32_t q;            /* must be QBX_Q                                          */
  const double* nodes;  /* device, [n_panels][16][2], counter-clockwise           */
} qbx_geometry;

/* ---- sizes ------------------------------------------------------------- */

/* Workspace bytes for qbx_layer_potential / _adjoint with these parameters
 * (0 if the parameters are invalid).  The size depends on the process-wide
 * tuning (qbx_set_tuning: the launch shapes set the number of partial sums),
 * so a workspace sized under one tuning can be too small under another, which
 * the entry points report as QBX_EWORKSPACE: query again after a tuning
 * change, or size for the largest shapes (qbx_autotune_workspace_bytes covers
 * every shape the autotuner tries, and more). */
size_t qbx_workspace_bytes(int n_panels, int q, int p, int oversample, int side, int kind);

/* Bytes of the forward's tape (the per-center data the adjoint reuses). */
size_t qbx_tape_bytes(int n_panels, int q, int p, int side, int kind);

/* ---- forward ----------------------------------------------------------- */

/* One-sided QBX limits of S sigma and/or D mu at every target.
 *   density [n_kinds][T] complex: the S density first, then the D density,
 *            sampled at the nodes (interpolated to the source grid inside).
 *   k > 0 wavenumber, p expansion order, r center distance as a fraction of the
 *   panel length, oversample source refinement, side, kind as above.
 *   out [n_sides][n_kinds][T] complex.
 *   tape: nullable device buffer of qbx_tape_bytes(); when given it receives
 *         what the adjoint needs so that it need not recompute it.       */
int qbx_layer_potential(const qbx_geometry* g, const double* density, double k, int p,
                        double r, int oversample, int side, int kind, double* out,
                        double* tape, void* ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the plain forward of
 * qbx_layer_potential (no tape), same arguments and results, with no
 * workspace.  Its scratch arrays live in a file-scope device array of
 * QBX_STATIC_SCRATCH_BYTES that every GPU the library runs on holds from the
 * module's load until the process ends; the call allocates and frees nothing.
 * The stream must belong to the current device.  All calls on one GPU share
 * that array, so calls that overlap on one GPU (other streams, other threads)
 * race: serialise them.  Errors as qbx_layer_potential, plus QBX_EWORKSPACE
 * when the problem needs more scratch than the array holds (about 64 MiB: for
 * example 1024 panels, oversample 4, one side, S, p = 16, fits; 4096 panels,
 * both sides, S+D does not) and QBX_EDEVICE when the array's address cannot be
 * looked up. */
#define QBX_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int qbx_layer_potential_noalloc(const qbx_geometry* g, const double* density, double k, int p,
                                double r, int oversample, int side, int kind, double* out,
                                hipStream_t stream);

/* Options of qbx_layer_potential_ext; zero-initialised, they are the defaults
 * of qbx_layer_potential. */
typedef struct {
  int32_t dipole;       /* 0: the D slot is the double layer (source derivative along
                           the outward normal); 1: it is the tangential dipole
                           R sigma(x) = int t(x') . grad_x' G(x, x') sigma(x') ds'
                           (eq. riesz-def), t the counter-clockwise unit tangent   */
  int32_t center_rule;  /* 0: center distance R = r h_m; 1: R = r sqrt(h_m), the
                           choice Section 3.1 names for an error that vanishes as
                           h -> 0 at fixed p                                       */
} qbx_forward_options;

/* qbx_layer_potential with the options above (opt may be NULL: the defaults).
 * R has no jump across the curve (R sigma = -S[d sigma/ds] by parts), so its two
 * one-sided limits agree up to the QBX error.  Forward only: the adjoint and
 * the tape assume the defaults.  QBX_EINVAL for an option outside {0, 1};
 * otherwise as qbx_layer_potential.  The workspace is qbx_workspace_bytes(). */
int qbx_layer_potential_ext(const qbx_geometry* g, const double* density, double k, int p,
                            double r, int oversample, int side, int kind,
                            const qbx_forward_options* opt, double* out, void* ws,
                            size_t ws_bytes, hipStream_t stream);

/* Target derivatives (Section 3.2: the local expansion at each center is
 * differentiated analytically with respect to the target), with the arguments
 * of qbx_layer_potential:
 *   grad  [n_sides][n_kinds][T][2] complex, nullable: (du/dx, du/dy), the
 *         one-sided limits of grad S sigma and grad D mu at every target;
 *   dn    [n_sides][n_kinds][T] complex, nullable: n . grad u, the one-sided
 *         limits of S' and D' (defined at the start of Section 4), n the
 *         outward unit normal at the target.
 * At least one of grad and dn must be given (QBX_EINVAL otherwise).  The
 * principal value of grad S (and of S') is the average of its two one-sided
 * limits (grad S = grad S^+- +- n sigma / 2); D' has no jump.  The pair pass
 * forms only q dK/dR and q dK/dtheta per center (launch shape of the forward
 * with tape).  Stream-ordered, no allocation; the workspace is
 * qbx_workspace_bytes(). */
int qbx_layer_potential_gradient(const qbx_geometry* g, const double* density, double k, int p,
                                 double r, int oversample, int side, int kind, double* grad,
                                 double* dn, void* ws, size_t ws_bytes, hipStream_t stream);

/* Near/far split of the forward (Section 5: QBX is needed only where a panel
 * is close to the target; distant panels are summed directly by a smooth
 * rule).  Source panel m' is near target panel m when
 *   |b_m - b_m'|^2 < gamma^2 max(rad2_m, rad2_m'),
 * b_m the mean of the panel's 16 nodes (added in node order, times 1/16) and
 * rad2_m = max_a |X_{m,a} - b_m|^2, every operation rounded on its own (no
 * fused multiply-add), so the decision is reproducible bit for bit.  Near
 * sources enter through the QBX expansion exactly as in qbx_layer_potential;
 * every other panel enters through its own 16-point Gauss-Legendre rule at its
 * nodes (weight w = omega |X'(tau)|, the node's normal, the node density, no
 * oversampling): each node x' adds (i/4) w sigma H_0(k|x - x'|) (S) or
 * (i/4) w mu dH_0(k|x - x'|)/dn' (D) at the target x itself.
 *   gamma > 0 (QBX_EINVAL otherwise); gamma^2 above the largest double makes
 *   every panel near, which is qbx_layer_potential.  Accuracy: the near
 *   sources alone form an open patch whose ends lie about gamma * sqrt(rad2)
 *   from the target, so the expansion adds an error near
 *   (r h / (gamma sqrt(rad2)))^(p+1); gamma = 6 suits p = 20, p = 10 needs
 *   about 16 for 1e-12.
 * Other arguments and out as qbx_layer_potential; no tape (the density
 * adjoint, qbx_layer_potential_split_adjoint, recomputes what it needs).
 * Stream-ordered, no allocation; the workspace is qbx_workspace_bytes(). */
int qbx_layer_potential_split(const qbx_geometry* g, const double* density, double k, int p,
                              double r, int oversample, int side, int kind, double gamma,
                              double* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Target derivatives with the near/far split: the outputs, arguments and
 * errors of qbx_layer_potential_gradient, plus gamma as in
 * qbx_layer_potential_split.  Near sources enter through the derivative of the
 * local expansion (Section 3.2); the others through the gradient of the
 * direct rule at the target, k H_1 and H_0 by the chain rule (shared by both
 * sides).  Stream-ordered, no allocation; qbx_workspace_bytes(). */
int qbx_layer_potential_split_gradient(const qbx_geometry* g, const double* density, double k,
                                       int p, double r, int oversample, int side, int kind,
                                       double gamma, double* grad, double* dn, void* ws,
                                       size_t ws_bytes, hipStream_t stream);

/* Vector-Jacobian product of qbx_layer_potential_split (PyTorch convention):
 * the gradients of L = Re <cotangent, out> with respect to the density (the
 * conjugate-transposed operator A^H applied to the cotangent) and, when
 * grad_nodes is not NULL, to the node coordinates.  The same near relation and
 * rules as the forward: each pair's term is differentiated under the rule it
 * takes (the QBX pair of Sections 2 and 3.2 for near pairs, the smooth rule for
 * far ones), through the source grid, weights, normals, centers, radii and the
 * targets themselves; the near relation is piecewise constant in the nodes and
 * contributes nothing.  <g, A sigma> = <A^H g, sigma> holds to rounding.
 *   cotangent     device, the shape of out
 *   grad_density  device [n_kinds][T] complex, or NULL
 *   grad_nodes    device [P][16][2], or NULL (density only: a cheaper path)
 * Errors as qbx_layer_potential_split, plus QBX_EINVAL for a NULL cotangent or
 * when both outputs are NULL.  Stream-ordered, no allocation;
 * qbx_workspace_bytes(). */
int qbx_layer_potential_split_adjoint(const qbx_geometry* g, const double* density, double k,
                                      int p, double r, int oversample, int side, int kind,
                                      double gamma, const double* cotangent,
                                      double* grad_density, double* grad_nodes, void* ws,
                                      size_t ws_bytes, hipStream_t stream);

/* ---- integral equation ------------------------------------------------ */

/* Workspace bytes of qbx_solve_dirichlet (0 for invalid arguments; side must
 * be -1 or 1, 1 <= restart <= 1000). */
size_t qbx_solve_workspace_bytes(int n_panels, int q, int p, int oversample, int side,
                                 int restart);

/* Nystrom solve of the Dirichlet problem by the combined-field representation
 * u = -D sigma + alpha S sigma (Section 4.3, eq. dirichlet-inteq):
 *   -+ sigma/2 + alpha S sigma - D sigma = f   at the nodes
 * (upper sign: side = 1, the exterior problem; side = -1 the interior one).
 * S and D are principal values, the averages of the two one-sided QBX limits
 * (eq. dlp-twosided): Section 3.5 shows that only the averaged D keeps the
 * spectral clustering that lets GMRES converge below the discretization error.
 * As in the paper the unknowns are sqrt(w) sigma (w the 16-point rule's weight
 * at the node) and GMRES(restart) iterates until the relative residual of that
 * scaled system is below tol (the paper uses 1e-14) or max_iter products have
 * been taken.  Each product is one S+D call for both sides of
 * qbx_layer_potential, or of qbx_layer_potential_split when gamma > 0
 * (gamma = 0: plain QBX).
 *   f      device [16 P] complex, the Dirichlet data at the nodes
 *   alpha  alpha_re + i alpha_im (the paper takes alpha = i)
 *   sigma  device [16 P] complex, out: the density
 *   iterations, residual: host, nullable; the matrix-vector products taken and
 *          the true relative residual |W^(1/2) (f - A sigma)| / |W^(1/2) f| of
 *          the returned sigma (check it: the call returns QBX_OK also when
 *          max_iter ends the iteration first).
 * SYNCHRONOUS on `stream` (the Arnoldi coefficients come back to the host after
 * every product).  No allocation; the workspace is qbx_solve_workspace_bytes().
 * Errors as qbx_layer_potential, plus QBX_EINVAL for side 0, restart, max_iter,
 * tol <= 0, gamma < 0 or a non-finite alpha. */
int qbx_solve_dirichlet(const qbx_geometry* g, const double* f, double k, int p, double r,
                        int oversample, int side, double alpha_re, double alpha_im, double gamma,
                        double tol, int restart, int max_iter, double* sigma, int* iterations,
                        double* residual, void* ws, size_t ws_bytes, hipStream_t stream);

/* The adjoint system of qbx_solve_dirichlet, (-+ 1/2 + conj(alpha) S^H - D^H)
 * lambda = rhs (S, D the same two-sided averages), by the same GMRES on
 * W^(-1/2) A^H W^(1/2); each product is one density adjoint for both sides
 * (qbx_layer_potential_adjoint, or qbx_layer_potential_split_adjoint when
 * gamma > 0).  For L = Re <g, sigma> with A sigma = f, lambda = A^-H g is the
 * gradient with respect to f, and -grad_x Re <lambda, A(x) sigma> the one with
 * respect to the nodes.  Arguments, workspace, errors and the synchronous
 * behaviour as qbx_solve_dirichlet; residual is that of the scaled adjoint
 * system. */
int qbx_solve_dirichlet_adjoint(const qbx_geometry* g, const double* rhs, double k, int p,
                                double r, int oversample, int side, double alpha_re,
                                double alpha_im, double gamma, double tol, int restart,
                                int max_iter, double* lambda, int* iterations, double* residual,
                                void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of qbx_solve_dirichlet_node_gradient (0 if invalid). */
size_t qbx_solve_node_gradient_workspace_bytes(int n_panels, int q, int p, int oversample);

/* Node part of the gradient through the solve.  For sigma = A(x)^-1 f (the
 * operator of qbx_solve_dirichlet) and a real loss L(sigma), the gradient
 * with respect to the nodes x is -grad_x Re <lambda, A(x) sigma> with sigma
 * held fixed and lambda = A^-H dL/dsigma (qbx_solve_dirichlet_adjoint).  The
 * -+ sigma/2 term does not depend on x, so this is one node adjoint of the
 * layer potentials (both sides, S and D, density sigma) with the cotangents
 * -conj(alpha) lambda / 2 for S and lambda / 2 for D on each side (the
 * averages of the two limits), formed on the device; the split's node
 * adjoint when gamma > 0.
 *   sigma, lambda  device [16 P] complex
 *   side           1 or -1, as for the solve (validated only)
 *   grad_nodes     device [P][16][2], out
 * Stream-ordered, no allocation; the workspace is
 * qbx_solve_node_gradient_workspace_bytes(). */
int qbx_solve_dirichlet_node_gradient(const qbx_geometry* g, const double* sigma,
                                      const double* lambda, double k, int p, double r,
                                      int oversample, int side, double alpha_re, double alpha_im,
                                      double gamma, double* grad_nodes, void* ws,
                                      size_t ws_bytes, hipStream_t stream);

/* ---- adjoint ----------------------------------------------------------- */

/* Vector-Jacobian product of qbx_layer_potential for the real scalar
 * L = Re sum conj(cotangent) * out (PyTorch convention):
 *   grad_density [n_kinds][T] complex = (d out / d density)^H cotangent,
 *   grad_nodes   [n_panels][16][2] real = dL/d nodes,
 * through every step: source interpolation, weights, normals, panel lengths,
 * centers, radii and the expansion sums.  cotangent has the layout of out.
 * tape: the forward's tape; the pair work is then one source-major pass.  With
 * tape NULL and grad_nodes wanted, one fused pass evaluates each pair once for
 * both gradient sides; with tape NULL and only grad_density wanted, only the
 * source-major pass runs.  Every path sums in a fixed order: repeated calls
 * give identical bits.  Either gradient pointer may be
 * NULL when not wanted.  The gradients are written, not accumulated. */
int qbx_layer_potential_adjoint(const qbx_geometry* g, const double* density, double k, int p,
                                double r, int oversample, int side, int kind,
                                const double* cotangent, const double* tape,
                                double* grad_density, double* grad_nodes, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* ---- batched: many contours in one persistent launch ---------------------- */

/* One contour of a batch.  Offsets locate its blocks inside the caller's packed
 * arrays (in units of panels for nodes and of complex values otherwise); the
 * blocks have the per-contour layouts of qbx_layer_potential:
 *   nodes   + node_offset*32    : [n_panels][16][2]
 *   density + 2*density_offset  : [n_kinds][16 n_panels] complex
 *   out     + 2*out_offset      : [n_sides][n_kinds][16 n_panels] complex
 * (cotangent, grad_density and grad_nodes of the adjoint use the layouts and
 * offsets of out, density and nodes).  Blocks of different contours must not
 * overlap.  All contours share `oversample`; p, k, r, side and kind are per
 * contour with the limits of qbx_layer_potential. */
typedef struct {
  int64_t node_offset;
  int64_t density_offset;
  int64_t out_offset;
  int32_t n_panels;
  int32_t p;
  int32_t kind;
  int32_t side;
  double k;
  double r;
} qbx_batch_item;

/* Workspace / tape bytes for a batch (items in HOST memory; 0 if invalid).
 * As for qbx_workspace_bytes, the workspace size depends on the tuning
 * (batch_adjoint_tasks, batch_fused_chunks): query again after a change. */
size_t qbx_batched_workspace_bytes(const qbx_batch_item* items, int n_items, int oversample);
size_t qbx_batched_tape_bytes(const qbx_batch_item* items, int n_items);

/* Forward for every contour of the batch.  The source grids and centers of all
 * contours are built by one launch; the pair work runs in one persistent launch
 * per (kind, p) class present in the batch (each compiled for its class), whose
 * wavefronts take (contour, center) tasks, most expensive contours first, from
 * the class's device counter.  The classes' launches are independent: they are
 * forked from `stream` onto up to three library streams of the current device
 * (default priority; created on the device's first batched call and kept until
 * the process ends) and joined back to `stream` with events, so that they
 * overlap and one class's tail is filled by the next.  The call stays ordered
 * on `stream` like every other; the stream must belong to the current device.
 * tape: nullable, the batch's tape for qbx_layer_potential_batched_adjoint
 * (qbx_batched_tape_bytes).  items is a HOST array; it is copied into the
 * workspace. */
int qbx_layer_potential_batched(const qbx_batch_item* items, int n_items, const double* nodes,
                                const double* density, double* out, double* tape, int oversample,
                                void* ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint of the batched forward (the per-contour qbx_layer_potential_adjoint
 * for every contour).  tape: the batched forward's tape; then the source-major
 * pass of all contours of a (kind, p) class runs in one persistent launch over
 * (contour, center split, 64-source chunk) tasks.  tape NULL with grad_nodes:
 * the fused pass, one persistent launch per class whose workgroups take
 * (contour, center block, source block) tiles; tape NULL with only
 * grad_density: the source-major pass alone.  The classes' launches overlap as
 * in the forward.  Reproducible bit for bit. */
int qbx_layer_potential_batched_adjoint(const qbx_batch_item* items, int n_items,
                                        const double* nodes, const double* density,
                                        const double* cotangent, const double* tape,
                                        double* grad_density, double* grad_nodes, int oversample,
                                        void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- stored local expansions: one center, several targets (Section 5) ------ */

/* Workspace bytes of qbx_expansion_coefficients (0 if the parameters are invalid). */
size_t qbx_expansion_workspace_bytes(int n_panels, int q, int p, int oversample, int side,
                                     int kind);

/* The local expansion coefficients of every center of the contour, formed once and
 * stored, so that a center's expansion can serve several nearby targets (Section 5
 * names this as an optimization): a_l, l = -p..p, of eq. graf-coefficient (S) and
 * eq. graf-coefficient-dlp (D), the same sums qbx_layer_potential evaluates at each
 * center's own target, without the factor i/4.
 *   coef   [n_kinds][Mc][2p+1] complex, index l + p; Mc = n_sides * T centers in
 *          the order of qbx_layer_potential's outputs (exterior first for BOTH)
 *   ctr_xy [Mc][2], ctr_r [Mc]: the centers and their radii (each nullable)
 * Arguments and errors as qbx_layer_potential; the workspace is
 * qbx_expansion_workspace_bytes. */
int qbx_expansion_coefficients(const qbx_geometry* g, const double* density, double k, int p,
                               double r, int oversample, int side, int kind, double* coef,
                               double* ctr_xy, double* ctr_r, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/* The stored expansions evaluated at any targets (Section 3.3, step 4(c), at a
 * target of the caller's choice):
 *   out[kind][t] = (i/4) sum_{l=-p..p} a_l J_l(k|x_t - c|) e^{i l arg(x_t - c)},
 * c = ctr_xy[center_index[t]], a the coefficients coef[kind][center_index[t]] of
 * qbx_expansion_coefficients (same n_ctr, p, kind).  The expansion converges for a
 * target closer to its center than every source; the center's disk (radius
 * ctr_r) holds such targets (qbx_assign_centers picks them).  A center index
 * outside [0, n_ctr) gives NaN.  target_xy [n_targets][2], center_index
 * [n_targets] (int32), out [n_kinds][n_targets] complex.  Stream-ordered, no
 * workspace.  QBX_EINVAL for bad sizes, p, k, kind or NULL arrays. */
int qbx_evaluate_expansions(int n_ctr, const double* ctr_xy, const double* coef, double k,
                            int p, int kind, int n_targets, const double* target_xy,
                            const int32_t* center_index, double* out, hipStream_t stream);

/* For every target, the nearest center whose disk holds it, |x_t - c| <= slack *
 * R_c (ties to the lower index), or -1 when no disk does.  ctr_xy [n_ctr][2],
 * ctr_r [n_ctr], target_xy [n_targets][2], center_index [n_targets] (int32, out).
 * Stream-ordered.  QBX_EINVAL for bad sizes, slack <= 0 or NULL arrays. */
int qbx_assign_centers(int n_ctr, const double* ctr_xy, const double* ctr_r, int n_targets,
                       const double* target_xy, double slack, int32_t* center_index,
                       hipStream_t stream);

/* ---- kernel level: explicit sources and centers ------------------------------ */

/* The QBX sums for sources and expansion centers given directly (no panels, no
 * interpolation): the pair loops of qbx_layer_potential applied to caller data,
 * e.g. one shard of the centers, or sources of another smooth rule.  For center
 * i at c_i with radius R_i and target direction e^{i theta_i} (its target is
 * x_i = c_i + R_i e^{i theta_i}):
 *   out[kind][i] = (i/4) sum_{l=-p..p} a_l J_l(k R_i) e^{i l theta_i},
 *   S: a_l = sum_j q_j H^(1)_l(k|x'_j - c_i|) e^{-i l theta'_ij}
 *      (Section 2, eq. graf-coefficient; Section 3.3 step 4(c)),
 *   D: the same with nu_j . grad_{x'_j} applied to the source factor
 *      (Section 3.2, eq. graf-coefficient-dlp), linear in the given normal nu_j.
 * Arguments (device arrays):
 *   src_xy  [n_src][2]            source points x'_j
 *   src_nu  [n_src][2]            source normals (D only; may be NULL for S)
 *   src_q   [n_kinds][n_src]      complex weighted densities q_j (quadrature weight
 *                                 times density), S first, then D
 *   ctr_xy  [n_ctr][2], ctr_r [n_ctr] (> 0), ctr_dir [n_ctr] complex unit e^{i theta}
 *   out     [n_kinds][n_ctr]      complex
 *   tape    nullable, qbx_explicit_tape_bytes(): per-center sums for the adjoint
 * The caller is responsible for Graf's condition |x_i - c_i| < |x'_j - c_i|.
 * Errors: QBX_EINVAL (n_src or n_ctr < 1, p, kind, k, NULL arrays, src_nu NULL
 * with D), QBX_EWORKSPACE, QBX_EDEVICE. */
size_t qbx_explicit_workspace_bytes(int n_src, int n_ctr, int p, int kind);
size_t qbx_explicit_tape_bytes(int n_ctr, int kind);
int qbx_apply_explicit(int n_src, const double* src_xy, const double* src_nu, const double* src_q,
                       int n_ctr, const double* ctr_xy, const double* ctr_r, const double* ctr_dir,
                       double k, int p, int kind, double* out, double* tape, void* ws,
                       size_t ws_bytes, hipStream_t stream);

/* Target derivatives of the same local expansions (Section 3.2: the expansion
 * about each center differentiated analytically in the target): the gradient
 * of out with respect to the target x_i = c_i + R_i e^{i theta_i}, the center
 * held fixed.  grad [n_kinds][n_ctr][2] complex (d/dx, d/dy).  The same pair
 * pass as qbx_layer_potential_gradient, on the caller's sources and centers:
 * with the source grid and centers of a contour it gives that entry point's
 * one-sided limits.  Errors as qbx_apply_explicit, plus QBX_EINVAL for a NULL
 * grad. */
int qbx_apply_explicit_gradient(int n_src, const double* src_xy, const double* src_nu,
                                const double* src_q, int n_ctr, const double* ctr_xy,
                                const double* ctr_r, const double* ctr_dir, double k, int p,
                                int kind, double* grad, void* ws, size_t ws_bytes,
                                hipStream_t stream);

/* Vector-Jacobian product of qbx_apply_explicit for L = Re sum conj(cotangent) out
 * (cotangent [n_kinds][n_ctr] complex); every gradient pointer is nullable and the
 * gradients are written, not accumulated:
 *   grad_q        [n_kinds][n_src] complex = (d out / d q)^H cotangent
 *   grad_src_xy   [n_src][2]   dL/dx'_j
 *   grad_src_nu   [n_src][2]   dL/d(nu_x, nu_y) (D; ignored without D)
 *   grad_ctr_xy   [n_ctr][2]   dL/dc_i with R_i and theta_i held (the target moves
 *                              with its center)
 *   grad_ctr_r    [n_ctr]      dL/dR_i
 *   grad_ctr_theta[n_ctr]      dL/dtheta_i (the direction as an angle)
 * tape: the forward's tape, or NULL to recompute it (needed for the center
 * gradients only). */
int qbx_apply_explicit_adjoint(int n_src, const double* src_xy, const double* src_nu,
                               const double* src_q, int n_ctr, const double* ctr_xy,
                               const double* ctr_r, const double* ctr_dir, double k, int p,
                               int kind, const double* cotangent, const double* tape,
                               double* grad_q, double* grad_src_xy, double* grad_src_nu,
                               double* grad_ctr_xy, double* grad_ctr_r, double* grad_ctr_theta,
                               void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- principal value (Section 3.2) --------------------------------------- */

/* pv [n_kinds][T] complex from out [n_sides][n_kinds][T] (the layout of
 * qbx_layer_potential's output for the same side and kind):
 *   side = QBX_BOTH: the average of the two one-sided limits (eq. dlp-twosided);
 *   one side s:      S is continuous across the curve, pv = out; for D the jump
 *                    relation (eq. dlpjump) gives pv = out - s*mu/2, with mu the
 *                    D density at the node (density [n_kinds][T], as given to the
 *                    forward; unused, may be NULL, when no D is present).
 * Stream-ordered, no allocation. */
int qbx_principal_value(const double* out, const double* density, int n_panels, int side,
                        int kind, double* pv, hipStream_t stream);

/* On-surface target derivatives from the one-sided limits of
 * qbx_layer_potential_gradient (or _split_gradient), by the jump relations of
 * Section 3.2 (x on the curve; + exterior, - interior):
 *   grad S(x) = grad S(x^+-) +- n sigma / 2   (principal value; S' = n . grad S
 *                                              jumps by sigma / 2 from each side)
 *   grad D(x) = grad D(x^+-) -+ t dmu/ds / 2  (finite part, eq. dlpderiv; D' has
 *                                              no jump)
 * with n the outward unit normal at the node and t = (-n_y, n_x) the
 * counter-clockwise unit tangent, both from the 16-node derivative of the panel
 * as for the centers, and dmu/ds the derivative along the curve of the
 * degree-15 interpolant of the D density through its 16 node values.
 *   side = QBX_BOTH: the average of the two limits (as eq. dlp-twosided does for
 *                    D); density unused, may be NULL.
 *   one side:        that limit minus its jump; density [n_kinds][T] as given to
 *                    the forward.
 *   grad [n_sides][n_kinds][T][2] complex -> grad_pv [n_kinds][T][2];
 *   dn   [n_sides][n_kinds][T] complex    -> dn_pv   [n_kinds][T].
 * Either pair may be NULL, not both; an input and its output are given together.
 * Stream-ordered, no allocation.  QBX_EINVAL for bad pointers, q, n_panels,
 * side or kind. */
int qbx_gradient_principal_value(const qbx_geometry* g, const double* density, int side,
                                 int kind, const double* grad, const double* dn, double* grad_pv,
                                 double* dn_pv, hipStream_t stream);

/* ---- checks ------------------------------------------------------------ */

/* SYNCHRONOUS geometry check (it waits for `stream`): signed area of the
 * contour and min over all centers and sources of |x'_j - c_i| / R_i.
 * Returns QBX_EORIENT if the area is negative, QBX_EGRAF if the minimum
 * ratio is below 1 - 1e-12, QBX_OK otherwise.  area / min_ratio (host, may be
 * NULL) receive the values. */
int qbx_check_geometry(const qbx_geometry* g, int p, double r, int oversample, int side,
                       double* area, double* min_ratio, void* ws, size_t ws_bytes,
                       hipStream_t stream);

/* Host-only signed area of a contour given in HOST memory, by the 16-point
 * panel rule; used to reject clockwise input without a GPU.  Returns
 * QBX_EINVAL for bad arguments, QBX_EORIENT if negative, else QBX_OK. */
int qbx_signed_area_host(const double* nodes_host, int n_panels, double* area);

/* ---- errors ------------------------------------------------------------ */

const char* qbx_strerror(int code);
const char* qbx_last_error(void);

/* ---- special functions (test hooks) ------------------------------------ */

/* H^(1)_0 and H^(1)_1 at n real points z > 0 exactly as the pair kernels
 * compute them: z, h0, h1 device arrays ([n], [n] complex, [n] complex). */
int qbx_debug_hankel01(const double* z, int n, double* h0, double* h1, hipStream_t stream);

/* J_0..J_L at n points x >= 0 by the Miller recurrence used for every center:
 * x [n], out [n][L+1]. L <= QBX_PMAX + 3. */
int qbx_debug_besselj(const double* x, int n, int L, double* out, hipStream_t stream);

/* ---- launch tuning and the autotuner --------------------------------------- */

/* Launch-shape parameters.  They change how the pair work is cut into
 * wavefront tasks (and so the order of the floating-point sums, nothing else).
 * Process-wide: every later call reads them.  Workspace sizes depend on them,
 * so query the *_workspace_bytes functions after changing them (a call whose
 * workspace became too small fails with QBX_EWORKSPACE).  Not thread-safe
 * against concurrent calls.
 *   forward_waves       per-contour plain forward: wavefronts aimed for per
 *                       launch; each center's source sum is split (in runs of
 *                       at least four 64-source chunks) until that many exist
 *   tape_waves          the same for the forward-with-tape kernel
 *   adjoint_waves       per-contour adjoint source pass: wavefronts aimed for;
 *                       the centers are split (at least 16 per split)
 *   batch_adjoint_tasks batched adjoint: tasks per (kind, p) class (64 sources
 *                       x a split of the centers, at least 16 centers each)
 *   batch_grid_scale    batched persistent kernels: workgroups launched =
 *                       workgroups resident on the device x this
 *   fused_tiles         adjoint without a tape: workgroup tiles (a block of
 *                       centers x a block of 64-source chunks) aimed for
 *   batch_fused_chunks  batched adjoint without a tape: 64-source chunks per tile
 *                       (four waves share a tile, one chunk each at a time)
 *   fused_part_bytes    adjoint without a tape (per contour and batched): bound
 *                       on its source-side partial sums, one row of sources per
 *                       tile of centers.  The tile height starts at 256 centers
 *                       and doubles while the rows would take more bytes; a
 *                       taller tile runs its centers in sub-blocks of 256.
 * Limits: the three wave targets, batch_adjoint_tasks and fused_tiles in
 * [256, 1 << 22], batch_grid_scale in [0.125, 8], batch_fused_chunks in
 * [1, 64], fused_part_bytes in [4096, 2^40].  Defaults 16384, 1.0, 16384, 4
 * and 2^31. */
typedef struct {
  int32_t forward_waves;
  int32_t tape_waves;
  int32_t adjoint_waves;
  int32_t batch_adjoint_tasks;
  double batch_grid_scale;
  int32_t fused_tiles;
  int32_t batch_fused_chunks;
  double fused_part_bytes;
} qbx_tuning;

/* Set / read the process-wide tuning (QBX_EINVAL for values out of range). */
int qbx_set_tuning(const qbx_tuning* t);
int qbx_get_tuning(qbx_tuning* t);

/* The passes an autotuner times (`fields`, a nonzero combination): */
#define QBX_TUNE_FORWARD 1   /* forward_waves; batched: batch_grid_scale */
#define QBX_TUNE_TAPE 2      /* tape_waves (the forward with tape) */
#define QBX_TUNE_ADJOINT 4   /* adjoint_waves; batched: batch_adjoint_tasks */
#define QBX_TUNE_FUSED 8     /* fused_tiles; batched: batch_fused_chunks */
#define QBX_TUNE_ALL 15

/* Workspace bytes of qbx_autotune (0 for invalid arguments): a workspace for
 * every candidate launch shape plus the output, tape and gradients it times. */
size_t qbx_autotune_workspace_bytes(int n_panels, int q, int p, int oversample, int side,
                                    int kind);

/* Autotuner for one contour problem (the arguments of qbx_layer_potential).
 * SYNCHRONOUS.  For each field selected in `fields` -- forward_waves,
 * tape_waves and adjoint_waves over 2048 .. 131072, fused_tiles over
 * 2048 .. 32768 (doubling; candidates that give the same launch shape are
 * timed once) -- it times its pass with hipEvents on `stream`, the minimum
 * over `passes` runs (1..20) after one warm-up, keeps the fastest, installs
 * the result with qbx_set_tuning and writes it to *best (nullable).  Other
 * fields are left as they were.  On error the previous tuning is restored.
 *   ws, ws_bytes  device workspace of qbx_autotune_workspace_bytes() bytes: all
 *                 device memory the timing uses (nothing is allocated)
 *   cache_path    host path of a text cache file, or NULL.  A line
 *                 "<key> => <value>" per result, the key naming the device
 *                 (architecture, compute units) and the problem (P, p,
 *                 oversample, side, kind, fields).  On a hit the stored fields
 *                 are installed untimed (ws may then be NULL); on a miss the
 *                 result is timed and written back (the file is rewritten
 *                 through a temporary file and a rename).  QBX_EIO for an
 *                 unreadable or unwritable file or a malformed entry; calls that
 *                 share a file from several processes at once may lose a line.
 */
int qbx_autotune(const qbx_geometry* g, const double* density, double k, int p, double r,
                 int oversample, int side, int kind, int passes, int fields,
                 const char* cache_path, qbx_tuning* best, void* ws, size_t ws_bytes,
                 hipStream_t stream);

/* Workspace bytes of qbx_autotune_batched (0 for an invalid batch). */
size_t qbx_autotune_batched_workspace_bytes(const qbx_batch_item* items, int n_items,
                                            int oversample);

/* Autotuner for a batch (the arguments of qbx_layer_potential_batched; items
 * in host memory, arrays on the device).  SYNCHRONOUS.  Times, as selected in
 * `fields`, batch_grid_scale in {0.5, 1, 2, 4} on the batched forward,
 * batch_adjoint_tasks in 2048 .. 262144 (doubling) on the batched adjoint
 * with the tape and batch_fused_chunks in {4, 8, 16, 32} on the batched
 * adjoint without it (QBX_TUNE_TAPE selects nothing here), keeps the fastest
 * of each and installs them.  ws, cache_path: as qbx_autotune, with
 * qbx_autotune_batched_workspace_bytes() and a key naming the device, the
 * item count, oversample, fields and a 64-bit signature of the items'
 * (n_panels, p, kind, side). */
int qbx_autotune_batched(const qbx_batch_item* items, int n_items, const double* nodes,
                         const double* density, int oversample, int passes, int fields,
                         const char* cache_path, qbx_tuning* best, void* ws, size_t ws_bytes,
                         hipStream_t stream);

/* ---- kernel timing (profiling hook) ----------------------------------- */

/* enable != 0: from now on every launch of a pair kernel (the forward and
 * adjoint hot loops) is bracketed by two hipEvents recorded on the caller's
 * stream; enable == 0 stops it and drops the records.  Host-side bookkeeping
 * only; not thread-safe. */
int qbx_kernel_timer(int enable);

/* SYNCHRONOUS: waits for the recorded events and returns, per kernel class
 * (0 = forward pair kernel, 1 = adjoint source pass, 2 = batched persistent
 * kernels, 3 = forward-with-tape pair kernel, 4 = fused adjoint pair kernel,
 * 5 = target-derivative pair kernel, 6 = near pass of the split forward,
 * 7 = far pass of the split forward, 8 = far pass of the split's density adjoint),
 * the summed duration in milliseconds and the number of launches since the
 * timer was enabled.  ms and launches are host arrays of QBX_TIMER_CLASSES. */
#define QBX_TIMER_CLASSES 9
int qbx_kernel_timer_read(double* ms, int* launches);

#ifdef __cplusplus
}
#endif
#endif /* QBX_H */
