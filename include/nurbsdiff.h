/*
 * nurbsdiff.h -- C ABI of libnurbsdiff, batched NURBS surface evaluation and
 * its adjoint on AMD Instinct MI355X (gfx950).
 *
 * The method is NURBS-Diff (arXiv 2104.14547).  The library evaluates
 *
 *     S(u,v) = sum_ij N_i^p(u) N_j^q(v) w_ij P_ij / sum_ij N_i^p(u) N_j^q(v) w_ij
 *
 * (Sec. 3.1.1, eq. NURBS) on tensor-product parameter grids, with the basis
 * from the Cox-de Boor recursion (eq. NURBSBasis, eq. BSplineBasis2), only
 * the p+1 (q+1) non-zero functions of each knot span (Sec. 3.1.2, steps 1-2)
 * and the homogeneous weighting and rational divide of Sec. 3.1.2 step 3.
 * The backward is the vector-Jacobian product of Sec. 3.2: dL/dP_ij by the
 * rational basis (eq. NURBSuDerivative4), dL/dw_ij (eq. NURBSvDerivative5)
 * and dL/dU_k, dL/dV_k through dS/dN_i (eq. NURBSvDerivative6) and the
 * knot derivative of the recursion (Sec. 3.2.1).  The Jacobian of
 * Sec. 3.2.2 is never formed.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All arrays are float32 in device memory unless stated otherwise.  The
 *    caller owns every buffer, including the workspace; the library never
 *    allocates on a hot-path call (plans allocate their tables once, at
 *    creation).  Outputs are fully overwritten, never accumulated.
 *  - Degrees: 1 <= p, q <= NURBS_MAX_DEGREE; control sides nu_c >= p+1,
 *    nv_c >= q+1.  Knot vectors have nu_c+p+1 (nv_c+q+1) entries, at most
 *    NURBS_MAX_KNOTS each (so nu_c <= NURBS_MAX_KNOTS-p-1), are
 *    non-decreasing, and satisfy U_p < U_{p+1} and U_{nu_c-1} < U_{nu_c}.
 *    nu_c * nv_c <= 2^26.  Weights are > 0.  Longer knot vectors return
 *    NURBS_EINVAL before anything is launched.
 *  - Knot spans are half-open, U_k <= u < U_{k+1}; a parameter equal to the
 *    last domain knot U_{nu_c} belongs to span nu_c-1.  Parameters are
 *    clamped into [U_p, U_{nu_c}] (the clamp carries no gradient).
 *  - Sample vectors us, vs must be non-decreasing (a tensor-product grid
 *    in the order it is stored).
 *  - An empty grid (nu_s or nv_s = 0, or B = 0) is valid: a forward writes
 *    nothing, a backward writes zero gradients.  The uniform-batch calls
 *    (nurbs_surface_*) then read no input array, so those may be NULL; in a
 *    ragged plan an empty surface is one entry among others.
 *  - Layouts (row-major): ctrl [nu_c][nv_c][3], w [nu_c][nv_c],
 *    ku [nu_c+p+1], kv [nv_c+q+1], us [nu_s], vs [nv_s],
 *    pts / grad_pts [nu_s][nv_s][3].
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    stream-ordered and asynchronous; none synchronises the host except
 *    nurbs_read_device_error.
 *  - Return codes: NURBS_OK (0) or a negative NURBS_E* code.  Errors that
 *    the host can detect are returned before anything is launched; the
 *    message is available from nurbs_last_error().  Data-dependent checks
 *    (knot order, weight sign, parameter domain, sample order) run on the
 *    device only with the NURBS_VALIDATE flag; without it such inputs are
 *    undefined behaviour (parameters outside the domain are clamped).
 *  - Results are deterministic: no floating-point atomics are used, and a
 *    surface's result does not depend on the other surfaces of its batch
 *    for a given tiling (nurbs_ctx_set_tiling): the tiling fixes the
 *    summation order of the backward.  Plans built with different tilings
 *    (for instance by an autotuner choosing per batch) agree within the
 *    FP32 tolerances, not bit for bit.
 */
#ifndef NURBSDIFF_H
#define NURBSDIFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NURBS_MAX_DEGREE 7
#define NURBS_MAX_KNOTS 256 /* entries per knot vector (staged whole in LDS) */

/* status codes */
#define NURBS_OK 0
#define NURBS_EINVAL -1       /* null pointer, bad shape, bad offset */
#define NURBS_EDEGREE -2      /* p, q outside [1, NURBS_MAX_DEGREE] or nu_c < p+1 */
#define NURBS_EKNOTS -3       /* (device, VALIDATE) knots decreasing or empty end span */
#define NURBS_EDOMAIN -4      /* (device, VALIDATE) sample outside the domain or unsorted */
#define NURBS_EWEIGHTS -5     /* (device, VALIDATE) a weight <= 0 */
#define NURBS_EWORKSPACE -6   /* workspace missing or too small */
#define NURBS_EDEVICE -7      /* HIP runtime error (text in nurbs_last_error) */
#define NURBS_EUNSUPPORTED -8 /* option not supported */

/* gradient selection for the backward */
#define NURBS_GRAD_CTRL 1u
#define NURBS_GRAD_W 2u
#define NURBS_GRAD_KU 4u
#define NURBS_GRAD_KV 8u
#define NURBS_GRAD_ALL 15u

/* flags */
#define NURBS_VALIDATE 1u /* run the device-side data checks */

/* bytes at the start of a plan's workspace that are not tile slots: the
 * error word and the dynamic schedule's tile counters (a plan forward needs
 * this much workspace under the dynamic schedule) */
#define NURBS_PLAN_WS_HEADER 4352

/* tile schedules of the ragged-batch plans (nurbs_ctx_set_schedule) */
#define NURBS_SCHED_STATIC 0  /* tiles assigned to waves when the plan is built (default) */
#define NURBS_SCHED_DYNAMIC 1 /* waves take tiles from counters at run time */

typedef struct nurbs_ctx nurbs_ctx;
typedef struct nurbs_plan nurbs_plan;

/* One surface of a ragged batch.  Offsets are element offsets (floats) into
 * the packed arrays passed to nurbs_plan_fwd / nurbs_plan_bwd.  Gradient
 * arrays reuse the offsets of the arrays they are gradients of (grad_ctrl at
 * ctrl_off, grad_w at w_off, grad_ku at ku_off, grad_kv at kv_off, grad_pts
 * at pts_off). */
typedef struct {
    int32_t p, q, nu_c, nv_c, nu_s, nv_s;
    int64_t ctrl_off, w_off, ku_off, kv_off, us_off, vs_off, pts_off;
} nurbs_desc;

/* ------------------------------------------------------------------------
 * Context.  Holds the device ordinal, flags and the last error text.  Not
 * thread-safe: one context per host thread.
 *   device : HIP device ordinal the calls run on (must be current).
 *   out    : receives the new context; release with nurbs_ctx_destroy.
 * ---------------------------------------------------------------------- */
int nurbs_ctx_create(int device, nurbs_ctx **out);
int nurbs_ctx_destroy(nurbs_ctx *ctx);
/* flags: NURBS_VALIDATE or 0; applies to the uniform-batch calls. */
int nurbs_ctx_set_flags(nurbs_ctx *ctx, unsigned flags);
/* Bandwidth of the Gaussian that smooths the degree-0 indicator's knot
 * derivative (Sec. 3.2.1).  Only sigma == 0, the zero-bandwidth limit in
 * which knot gradients are the exact derivative of the piecewise-polynomial
 * basis, is supported; any other value returns NURBS_EUNSUPPORTED. */
int nurbs_ctx_set_knot_sigma(nurbs_ctx *ctx, float sigma);
/* Tiling of later calls on this context: the target number of sample points
 * per forward / backward tile (a tile is one wave over <= 64 sample columns
 * and as many rows as reach the target; 0 restores the default, 16384).
 * Results stay bitwise reproducible for a given tiling; different tilings
 * change the summation order of the backward within the tolerances.  An
 * autotuner picks these per workload. */
int nurbs_ctx_set_tiling(nurbs_ctx *ctx, int fwd_tile_points, int bwd_tile_points);
/* How plans created later on this context hand tiles to their persistent
 * waves (Alg. Forward / Alg. Backward run all tiles in parallel; this is
 * only their order on the GPU):
 *   NURBS_SCHED_STATIC  : each wave runs a list fixed when the plan is built
 *                         (longest-processing-time greedy on a cost model);
 *                         the default;
 *   NURBS_SCHED_DYNAMIC : the tiles are ordered by decreasing estimated cost
 *                         and dealt to 16 queues; each wave runs one tile of
 *                         its queue and then takes the next from the queue's
 *                         counter in the workspace header (one integer
 *                         atomic per tile).  Plan forwards then need
 *                         NURBS_PLAN_WS_HEADER bytes of workspace.
 * Both give bit-identical results (every tile writes its own slot).
 * NURBS_EINVAL for any other value. */
int nurbs_ctx_set_schedule(nurbs_ctx *ctx, int schedule);
const char *nurbs_status_string(int status);
/* Text of the last error raised on this context (never NULL). */
const char *nurbs_last_error(nurbs_ctx *ctx);
/* Number of compute units of the context's device (for callers sizing work). */
int nurbs_ctx_device_info(nurbs_ctx *ctx, int *num_cus, int *wave_size);

/* ------------------------------------------------------------------------
 * Uniform batch: B surfaces of identical shape -- the paper's call
 * surface(ctrl, weights, knot_u, knot_v, p, q, uv) -> points (Sec. 3.1,
 * Alg. Forward; Sec. 3.2, Alg. Backward).
 *   ctrl [B][nu_c][nv_c][3], w [B][nu_c][nv_c], ku [B][nu_c+p+1],
 *   kv [B][nv_c+q+1]; us [nu_s], vs [nv_s] if uv_shared != 0 else
 *   us [B][nu_s], vs [B][nv_s]; pts [B][nu_s][nv_s][3].
 *   ws / ws_bytes : caller-owned device workspace of at least the size
 *   reported by nurbs_surface_ws_bytes (with the same shapes and mask);
 *   may be NULL when that size is 0.
 * ---------------------------------------------------------------------- */
int nurbs_surface_ws_bytes(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                           int nu_s, int nv_s, unsigned grad_mask, size_t *out);

int nurbs_surface_fwd(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                      const float *ctrl, const float *w, const float *ku,
                      const float *kv, int nu_s, int nv_s, const float *us,
                      const float *vs, int uv_shared, float *pts, void *ws,
                      size_t ws_bytes, void *stream);

/* Parametric derivatives and unit normals on the same grid (Appendix A,
 * eq. NURBSuDerivative1: S_u = (A_u - S w_u) / w, with A the homogeneous
 * point sum and A_u its sum over dN_i/du; S_v likewise), the quantities
 * surface offsetting moves points along (Sec. 4.3).  Inputs as
 * nurbs_surface_fwd.  Outputs, each [B][nu_s][nv_s][3] and each optional
 * (NULL: not computed, at least one must be given):
 *   pts     : S (the same values as nurbs_surface_fwd up to the last ulp of
 *             the divide);
 *   pts_du  : dS/du;   pts_dv : dS/dv;
 *   normals : (S_u x S_v) / |S_u x S_v|, and (0, 0, 0) where S_u x S_v = 0.
 * The derivatives are one-sided at knots: they are those of the span the
 * parameter falls in (half-open spans, the last one closed).  No workspace
 * is needed except under NURBS_VALIDATE (256 bytes for the error word). */
int nurbs_surface_derivs(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                         const float *ctrl, const float *w, const float *ku,
                         const float *kv, int nu_s, int nv_s, const float *us,
                         const float *vs, int uv_shared, float *pts, float *pts_du,
                         float *pts_dv, float *normals, void *ws, size_t ws_bytes,
                         void *stream);

/* Vector-Jacobian product.  grad_pts = dL/dS [B][nu_s][nv_s][3].  Outputs
 * (each overwritten when its grad_mask bit is set, untouched and allowed to
 * be NULL otherwise): grad_ctrl [B][nu_c][nv_c][3], grad_w [B][nu_c][nv_c],
 * grad_ku [B][nu_c+p+1], grad_kv [B][nv_c+q+1].  No gradient is returned
 * for the parameters us, vs (the paper's module does not use dS/du). */
int nurbs_surface_bwd(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                      const float *ctrl, const float *w, const float *ku,
                      const float *kv, int nu_s, int nv_s, const float *us,
                      const float *vs, int uv_shared, const float *grad_pts,
                      float *grad_ctrl, float *grad_w, float *grad_ku,
                      float *grad_kv, unsigned grad_mask, void *ws,
                      size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Fixed knots: the B-spline layer with a precomputed basis (Appendix E's
 * layer whose basis is computed once; the fixed-knot fits of Sec. 4.2).
 * While the knots and samples do not change, the span and the p+1 basis
 * values of every sample are computed once into a table and the grid calls
 * below read them instead of searching and evaluating the recursion.
 * Knot gradients are not available on these calls (the knots are fixed).
 *
 * Table layout (device memory, caller-owned): int32 spans [nx], then, at
 * the next multiple of 256 bytes, float basis [nx][p+1]; the same values
 * nurbs_find_spans and nurbs_basis return.
 * ---------------------------------------------------------------------- */
int nurbs_basis_table_bytes(int p, int nx, size_t *out);
/* Fills `table` for parameters x [nx] on the knot vector knots [n_knots]
 * (n_knots <= NURBS_MAX_KNOTS).  NURBS_EWORKSPACE if table_bytes is below
 * nurbs_basis_table_bytes(p, nx). */
int nurbs_basis_table_build(const float *knots, int n_knots, int p, const float *x, int nx,
                            void *table, size_t table_bytes, void *stream);

/* nurbs_surface_fwd / nurbs_surface_bwd with the tables of the u samples
 * (degree p, nu_s samples) and the v samples (degree q, nv_s samples):
 * tab_shared != 0: one pair of tables for the whole batch (every surface
 * has the same knots and samples); else B tables each, back to back with a
 * stride of nurbs_basis_table_bytes.  The tables must have been built from
 * the ku, kv, us, vs passed here (which the kernels still stage).  The
 * backward's grad_mask takes NURBS_GRAD_CTRL and NURBS_GRAD_W only;
 * workspace as nurbs_surface_ws_bytes with that mask.  Results equal those
 * of the calls without tables bit for bit. */
int nurbs_surface_fwd_tab(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                          const float *ctrl, const float *w, const float *ku,
                          const float *kv, int nu_s, int nv_s, const float *us,
                          const float *vs, int uv_shared, const void *tab_u,
                          const void *tab_v, int tab_shared, float *pts, void *ws,
                          size_t ws_bytes, void *stream);
int nurbs_surface_bwd_tab(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                          const float *ctrl, const float *w, const float *ku,
                          const float *kv, int nu_s, int nv_s, const float *us,
                          const float *vs, int uv_shared, const void *tab_u,
                          const void *tab_v, int tab_shared, const float *grad_pts,
                          float *grad_ctrl, float *grad_w, unsigned grad_mask, void *ws,
                          size_t ws_bytes, void *stream);

/* The same backward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument; the tile slots live in a 64 MiB array
 * that the library keeps in device memory (one per device it runs on, held
 * until the process ends).  Arguments, outputs and results as
 * nurbs_surface_bwd, bit for bit.
 * Limits and errors: NURBS_EWORKSPACE when the shapes need more than the
 * 64 MiB that nurbs_surface_ws_bytes would report (use nurbs_surface_bwd
 * with a workspace then); NURBS_EUNSUPPORTED under NURBS_VALIDATE (no data
 * checks here); NURBS_EINVAL when the context's device is not current at
 * the first call on that device.  The call itself allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).
 * Concurrency: every call on a device shares that device's array, so calls
 * that overlap on one device (different streams, or different threads
 * without ordering) race and give wrong results; serialise them (one
 * stream, or events).  The array keeps the last call's contents. */
int nurbs_surface_bwd_noalloc(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                              const float *ctrl, const float *w, const float *ku,
                              const float *kv, int nu_s, int nv_s, const float *us,
                              const float *vs, int uv_shared, const float *grad_pts,
                              float *grad_ctrl, float *grad_w, float *grad_ku,
                              float *grad_kv, unsigned grad_mask, void *stream);

/* ------------------------------------------------------------------------
 * Surfaces at scattered parameter pairs: eq. NURBS at each (u_k, v_k), in
 * any order (Sec. 3.1 evaluates the grid of all pairs of two lists; a
 * point cloud with its own parameters needs single pairs).  B surfaces of
 * one shape, npts pairs each:
 *   ctrl [B][nu_c][nv_c][3], w [B][nu_c][nv_c], ku [B][nu_c+p+1],
 *   kv [B][nv_c+q+1]; uv [npts][2] if uv_shared else [B][npts][2];
 *   pts, pts_du, pts_dv, grad_pts [B][npts][3].
 * Shape, knot, weight and parameter rules as for the grids (parameters
 * clamped into the domain, half-open spans); the pairs need not be sorted.
 * Workspace: nurbs_surface_uv_ws_bytes (0 for a forward without
 * NURBS_VALIDATE).
 * ---------------------------------------------------------------------- */
int nurbs_surface_uv_ws_bytes(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                              int npts, unsigned grad_mask, size_t *out);

/* S at every pair and, for each non-NULL one of pts_du, pts_dv, the
 * parametric derivatives (Appendix A, eq. NURBSuDerivative1).  At least
 * one output must be given. */
int nurbs_surface_uv_fwd(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                         const float *ctrl, const float *w, const float *ku,
                         const float *kv, int npts, const float *uv, int uv_shared,
                         float *pts, float *pts_du, float *pts_dv, void *ws,
                         size_t ws_bytes, void *stream);

/* Vector-Jacobian product at the pairs (Sec. 3.2 at each pair); outputs
 * and grad_mask as nurbs_surface_bwd.  Each gradient entry is a sum over
 * pairs in arbitrary order, so the terms are added exactly: each is rounded
 * to a multiple of 2^-s (2^s the largest power of two with npts times the
 * largest term of that gradient tensor at most 2^62) and summed as 64-bit
 * integers, which is order-independent (bitwise reproducible, no float
 * atomics).  The rounding adds at most npts * max|term| * 2^-63 per entry. */
int nurbs_surface_uv_bwd(nurbs_ctx *ctx, int B, int p, int q, int nu_c, int nv_c,
                         const float *ctrl, const float *w, const float *ku,
                         const float *kv, int npts, const float *uv, int uv_shared,
                         const float *grad_pts, float *grad_ctrl, float *grad_w,
                         float *grad_ku, float *grad_kv, unsigned grad_mask, void *ws,
                         size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Curves: B rational B-spline curves of one shape in the plane (dim 2) or in
 * space (dim 3),
 *     C(u) = sum_i N_i^p(u) w_i P_i / sum_i N_i^p(u) w_i,
 * eq. NURBS with one parametric direction (Sec. 3 builds curves from the
 * surface formulas by dropping a direction; the curve fits of Sec. 4.1).
 *   ctrl [B][nc][dim], w [B][nc], knots [B][nc+p+1]; us [ns] if u_shared
 *   else [B][ns]; pts, pts_du, grad_pts [B][ns][dim].
 * Degree, knot, weight and parameter rules are those of the surface calls
 * with one direction (1 <= p <= NURBS_MAX_DEGREE, nc >= p+1,
 * nc+p+1 <= NURBS_MAX_KNOTS, clamped parameters, half-open spans).  The
 * parameters need not be sorted; sorted ones take the faster reduction.
 * Workspace: nurbs_curve_ws_bytes; 0 bytes for a forward without
 * NURBS_VALIDATE; the backward needs at least the 256-byte header, plus one
 * partial per 2048 samples for curves with more samples than that.
 * ---------------------------------------------------------------------- */
int nurbs_curve_ws_bytes(nurbs_ctx *ctx, int B, int p, int nc, int dim, int ns,
                         unsigned grad_mask, size_t *out);

/* Points C(u) and, when pts_du is not NULL, the tangents dC/du
 * (eq. NURBSuDerivative1 with one direction: (A_u - C W_u) / W). */
int nurbs_curve_fwd(nurbs_ctx *ctx, int B, int p, int nc, int dim, const float *ctrl,
                    const float *w, const float *knots, int ns, const float *us,
                    int u_shared, float *pts, float *pts_du, void *ws, size_t ws_bytes,
                    void *stream);

/* Vector-Jacobian product (Sec. 3.2 with one direction): grad_pts = dL/dC.
 * grad_mask bits NURBS_GRAD_CTRL, NURBS_GRAD_W and NURBS_GRAD_KU (the knot
 * vector); NURBS_GRAD_KV is rejected.  Outputs as for the surfaces:
 * grad_ctrl [B][nc][dim], grad_w [B][nc], grad_knots [B][nc+p+1], each
 * overwritten when its bit is set.  Deterministic (no atomics). */
int nurbs_curve_bwd(nurbs_ctx *ctx, int B, int p, int nc, int dim, const float *ctrl,
                    const float *w, const float *knots, int ns, const float *us,
                    int u_shared, const float *grad_pts, float *grad_ctrl,
                    float *grad_w, float *grad_knots, unsigned grad_mask, void *ws,
                    size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Point-set losses: the Chamfer and Hausdorff distances of Sec. 4
 * (eqs. ChamferDistance and HausdorffDistance), two-sided, with the
 * Euclidean norm, between evaluated points P and a target set Q, for B
 * pairs of sets of equal sizes:
 *     CD = sum_i min_j |P_i - Q_j| + sum_j min_i |P_i - Q_j|
 *     HD = max_i min_j |P_i - Q_j| + max_j min_i |P_i - Q_j|
 *   P [B][n][dim], Q [B][m][dim] (dim 2 or 3), n, m >= 1, m <= 2^22.
 * Nearest and farthest points are integer decisions taken in float32 on
 * the float32 inputs with d2 = fma(dz, dz, fma(dy, dy, dx * dx)) (dz = 0
 * in the plane): the smallest d2 wins with the first index on ties, the
 * largest d2 wins with the first index on ties.  Squared distances must be
 * finite.  Distances and sums are then FP64, returned as float32.
 * Workspace: nurbs_chamfer_ws_bytes (covers both calls below).
 * ---------------------------------------------------------------------- */
int nurbs_chamfer_ws_bytes(nurbs_ctx *ctx, int B, int n, int m, size_t *out);

/* For each X[b][i] the index idx[b][i] of its nearest point in Y[b] and
 * that squared distance d2[b][i] (int32 and float32, device arrays
 * [B][n]).  Brute force over all pairs.  ws: at least the size that
 * nurbs_chamfer_ws_bytes(ctx, B, n, m) reports (small query sets split the
 * target set over several workgroups and keep per-range partials there);
 * NURBS_EWORKSPACE otherwise. */
int nurbs_nearest(nurbs_ctx *ctx, int B, int dim, const float *X, int n, const float *Y,
                  int m, int32_t *idx, float *d2, void *ws, size_t ws_bytes, void *stream);

/* out [B][2] = (CD, HD) per pair (device); grad_cd, grad_hd [B][n][dim]:
 * their gradients with respect to P (either may be NULL):
 *   dCD/dP_i = u(P_i, Q_a(i)) + sum over j with b(j) = i of u(P_i, Q_j)
 *   dHD/dP_i = [i = i*] u(P_i, Q_a(i)) + [i = b(j*)] u(P_i, Q_j*)
 * with u(x, y) = (x - y)/|x - y| (0 when x = y), a / b the nearest maps
 * and i*, j* the farthest points of P and Q.  Bitwise reproducible: the
 * sum over the targets that chose a point is kept in 2^-40 fixed point with
 * 64-bit integer adds (exact, order-independent); no float atomics. */
int nurbs_chamfer(nurbs_ctx *ctx, int B, int dim, const float *P, int n, const float *Q,
                  int m, float *out, float *grad_cd, float *grad_hd, void *ws,
                  size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Ragged batch ("plan"): thousands of surfaces of uneven degree, control
 * grid and sample grid in one persistent launch per direction (the paper's
 * batched forward of Alg. Forward over all surfaces, and Alg. Backward).
 *   host     : n descriptors in host memory (copied; may be freed after).
 *   flags    : NURBS_VALIDATE or 0.
 *   out      : receives the plan (owns its device tables).
 *   ws_bytes : receives the workspace size the plan's calls need.
 * The plan is bound to the device current at creation.  nurbs_plan_fwd /
 * nurbs_plan_bwd take packed arrays laid out as the descriptors say, launch
 * without host synchronisation or allocation, and may be captured in a HIP
 * graph.  Tiles are assigned to the persistent waves when the plan is built
 * (no device-side work queue), so calls of one plan on different streams may
 * overlap as long as each has its own workspace and outputs; the host-side
 * calls themselves are not thread-safe (one thread per plan).
 * ---------------------------------------------------------------------- */
int nurbs_plan_create(nurbs_ctx *ctx, const nurbs_desc *host, int n, unsigned flags,
                      nurbs_plan **out, size_t *ws_bytes);
/* The same plan with its device tables in caller memory, for loops that must
 * neither allocate nor synchronise (a serving loop building one plan per
 * batch of requests).
 *   tables, tables_bytes : device memory for the tables (at least
 *                 *table_bytes_needed bytes, 256-byte aligned).  NULL: size
 *                 query only; table_bytes_needed and ws_bytes are filled and
 *                 no plan is created (out may be NULL).
 *   stream      : the tables are uploaded with an asynchronous copy on this
 *                 stream; use the plan on it (or after it).
 * The plan does not own `tables`; nurbs_plan_destroy frees only host state.
 * Destroy the plan, and reuse `tables`, only after the stream has passed the
 * plan's last launch.  Errors as nurbs_plan_create, and NURBS_EWORKSPACE when
 * tables_bytes is too small. */
int nurbs_plan_create_in(nurbs_ctx *ctx, const nurbs_desc *host, int n, unsigned flags,
                         void *tables, size_t tables_bytes, void *stream,
                         nurbs_plan **out, size_t *table_bytes_needed, size_t *ws_bytes);
int nurbs_plan_destroy(nurbs_plan *plan);
/* Tile statistics of a plan: number of forward / backward tiles. */
int nurbs_plan_info(nurbs_plan *plan, int *fwd_tiles, int *bwd_tiles, int *grid);

/* ws / ws_bytes: the plan's workspace (at least the reported size for the
 * backward; for a forward, NURBS_PLAN_WS_HEADER bytes under the dynamic
 * schedule -- its tile counters -- or 256 under NURBS_VALIDATE -- the error
 * word).  Calls that may overlap need workspaces of their own. */
int nurbs_plan_fwd(nurbs_plan *plan, const float *ctrl, const float *w,
                   const float *ku, const float *kv, const float *us,
                   const float *vs, float *pts, void *ws, size_t ws_bytes,
                   void *stream);

int nurbs_plan_bwd(nurbs_plan *plan, const float *ctrl, const float *w,
                   const float *ku, const float *kv, const float *us,
                   const float *vs, const float *grad_pts, float *grad_ctrl,
                   float *grad_w, float *grad_ku, float *grad_kv,
                   unsigned grad_mask, void *ws, size_t ws_bytes, void *stream);

/* Kernel timing of plan calls (tracing).  With max_calls > 0, every later
 * nurbs_plan_fwd / nurbs_plan_bwd records HIP events around its kernels on
 * the call's stream, in a ring of max_calls slots per direction; 0 turns it
 * off.  The events are created here, never on a hot-path call.  Leave it off
 * while capturing a graph. */
int nurbs_plan_set_timing(nurbs_plan *plan, int max_calls);
/* Waits for the recorded events and returns, per recorded call, the kernel
 * durations in milliseconds: fwd[i] the forward kernel; bwd[i] the backward
 * row-loop kernel, gat[i] its gather kernel (the v-contraction of the tile
 * accumulators into dL/dPw rectangles; about 0 when neither dL/dP nor dL/dw
 * was asked for) and fin[i] the finalize kernel of backward call i.  Arrays
 * hold at least max_calls entries (any may be NULL); *n_fwd / *n_bwd receive
 * the number of entries written (the most recent calls, oldest first). */
int nurbs_plan_read_timing(nurbs_plan *plan, float *fwd, int *n_fwd, float *bwd, float *gat,
                           float *fin, int *n_bwd);

/* ------------------------------------------------------------------------
 * Test exports: the device span search and basis used by the kernels.
 *   knots [n_knots] (device), x [nx] (device); p in [1, NURBS_MAX_DEGREE].
 *   spans [nx] int32 (device): k with U_k <= x < U_{k+1} (Sec. 3.1.2 step 1,
 *   half-open, last span closed; x clamped into the domain).
 *   N [nx][p+1] (device): N_{k-p..k}^p(x) (eq. NURBSBasis).
 * ---------------------------------------------------------------------- */
int nurbs_find_spans(const float *knots, int n_knots, int p, const float *x, int nx,
                     int32_t *spans, void *stream);
int nurbs_basis(const float *knots, int n_knots, int p, const float *x, int nx,
                float *N, void *stream);

/* Synchronises `stream`, reads the first data error recorded by a
 * NURBS_VALIDATE call into its workspace `ws`, stores it in *code
 * (NURBS_OK if none) and clears it. */
int nurbs_read_device_error(const void *ws, void *stream, int *code);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of evaluation + gradient requests on
 * resident surfaces, in native threads.  A request names a resident surface
 * and brings a parameter grid (us, vs) and target points T; it receives S on
 * the grid (Sec. 3.1, eq. NURBS) and the gradients of
 * L = sum_ab ||S(u_a, v_b) - T_ab||^2 with respect to the surface's control
 * points, weights and knot vectors (Sec. 3.2: eq. NURBSuDerivative4,
 * eq. NURBSvDerivative5, eq. NURBSvDerivative6), computed as one ragged plan
 * per batch of requests.
 *
 * Batches: requests are taken in arrival order while the batch fits a slot's
 * device memory and fewer than max_requests are taken; a request for a
 * surface already in the forming batch stays queued for a later batch (its
 * gradients would land at the same offsets); the first request that does not
 * fit ends the batch.  Each of n_slots slots has its own stream, device
 * arena of slot_bytes and pinned host buffer of slot_bytes, so up to n_slots
 * batches are in flight.  A request's result does not depend on the other
 * requests of its batch, bit for bit (the plan's tiles follow each surface's
 * own shape; the tiling is the context default).
 * ---------------------------------------------------------------------- */
typedef struct nurbs_server nurbs_server;

/*   device      : HIP device ordinal.
 *   pool        : n_surf descriptors (host, copied): p, q, nu_c, nv_c and
 *                 ctrl_off, w_off, ku_off, kv_off into the resident arrays;
 *                 the sample fields are ignored.
 *   ctrl, w, ku, kv : the resident surfaces (device), packed as `pool` says;
 *                 the caller keeps them alive and unchanged until
 *                 nurbs_server_destroy.
 *   n_slots     : batches in flight, 1..16; max_requests 1..65536 per batch;
 *                 slot_bytes >= 64 KiB.
 * Allocates n_slots * (2 slot_bytes + the pool's gradient arrays) of device
 * and pinned host memory and starts the engine and completion threads. */
int nurbs_server_create(int device, const nurbs_desc *pool, int n_surf, const float *ctrl,
                        const float *w, const float *ku, const float *kv, int n_slots,
                        size_t slot_bytes, int max_requests, nurbs_server **out);
/* Queues one request; thread-safe.
 *   us [nu_s], vs [nv_s], target [nu_s][nv_s][3] : host memory, read when
 *                 the request's batch is packed;
 *   out         : host memory of 3 nu_s nv_s + 4 nu_c nv_c + (nu_c+p+1) +
 *                 (nv_c+q+1) floats, written when the batch completes:
 *                 S [nu_s][nv_s][3], dL/dP [nu_c][nv_c][3], dL/dw [nu_c][nv_c],
 *                 dL/dU [nu_c+p+1], dL/dV [nv_c+q+1];
 *   The caller owns all five buffers and keeps them until
 *   nurbs_server_wait(id) has returned (or the server is destroyed).
 *   t_arrival   : latency origin in seconds of CLOCK_MONOTONIC; < 0: now.
 *   id          : receives the request id (ids count up from 0).
 * NURBS_EINVAL for a bad surface index, NULL buffer or empty grid;
 * NURBS_EWORKSPACE when the request alone does not fit a slot; no id is
 * issued then. */
int nurbs_server_submit(nurbs_server *srv, int surf, const float *us, int nu_s, const float *vs,
                        int nv_s, const float *target, float *out, double t_arrival, int64_t *id);
/* Blocks until request `id` has finished; returns NURBS_OK or the error of
 * its batch (text in nurbs_server_last_error) and its latency in seconds
 * (arrival to the moment its batch's results were copied out). */
int nurbs_server_wait(nurbs_server *srv, int64_t id, double *latency);
/* Batches launched, requests finished, and the lowest id not yet finished
 * (every id below it has finished). */
int nurbs_server_stats(nurbs_server *srv, int64_t *batches, int64_t *completed,
                       int64_t *finished_below);
/* Host time, in seconds, the engine thread spent forming, packing and
 * launching batches and the completion thread spent copying results out
 * (waits excluded): where a saturated server's host time goes. */
int nurbs_server_busy(nurbs_server *srv, double *engine_s, double *completion_s);
const char *nurbs_server_last_error(nurbs_server *srv);
/* Serves every queued request, stops the threads and frees the slots. */
int nurbs_server_destroy(nurbs_server *srv);
/* The batch-formation rule alone (host logic, no device): n queued requests
 * in arrival order with their surfaces and device bytes; a batch has
 * fixed_bytes besides its requests' and holds at most max_requests.  Writes
 * the indices taken, ascending, to take[0..*n_take).  At most
 * 4 max_requests requests are passed over for a surface already taken. */
int nurbs_server_admit(const int32_t *surf, const size_t *nbytes, int n, size_t capacity,
                       size_t fixed_bytes, int max_requests, int32_t *take, int *n_take);

#ifdef __cplusplus
}
#endif
#endif /* NURBSDIFF_H */
