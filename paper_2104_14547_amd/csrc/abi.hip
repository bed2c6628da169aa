// libnurbsdiff host side: the C ABI of include/nurbsdiff.h.  Validates
// arguments, builds tilings and ragged-batch plans, and launches the kernels
// of the k_*.hip translation units on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "../../include/nurbsdiff.h"
#include "kernels.hpp"
#include "launch.hpp"

using namespace nd;

struct nurbs_ctx {
    int device = 0;
    unsigned flags = 0;
    int num_cus = 0;
    int occ[2][2] = {{0, 0}, {0, 0}};  // persistent-kernel workgroups per CU: [class d5, d7][fwd, bwd]
    int fwd_tile_pts = 16384;          // target points per forward / backward tile
    int bwd_tile_pts = 16384;
    int schedule = NURBS_SCHED_STATIC;  // of plans created on this context
    std::string err;
};

struct nurbs_plan {
    nurbs_ctx* ctx = nullptr;
    int device = 0;
    int n = 0;
    unsigned flags = 0;
    std::vector<nurbs_desc> host;
    // device tables (one allocation)
    void* dev = nullptr;
    DevDesc* d_desc = nullptr;
    DevTile* d_ftiles = nullptr;
    ExecTile* d_fexec = nullptr;  // forward execution records, wave order
    DevTile* d_btiles = nullptr;
    ExecTile* d_bexec = nullptr;  // backward execution records, wave order
    ExecTile* d_gexec = nullptr;  // backward records by decreasing estimated gather work
    int* d_fbegin = nullptr;      // wave boundaries in d_fexec
    int* d_bbegin = nullptr;      // wave boundaries in d_bexec
    int2* d_fin = nullptr;        // finalize parts (surface, part), most expensive first
    int nfin = 0;
    int nf = 0, nb = 0;
    int grid_fwd = 0, grid_bwd = 0;
    size_t ws_bytes = 0;
    int max_nU = 0, max_nV = 0;
    int maxd = 5;  // degree class of the persistent kernels (5 or 7)
    int schedule = NURBS_SCHED_STATIC;
    std::vector<char> staging;  // host copy of the tables (plans made in caller memory)
    // tracing: event ring per direction (2 events per forward, 4 per backward)
    int trace_slots = 0;
    std::vector<hipEvent_t> ev_f, ev_b;
    long long calls_f = 0, calls_b = 0;
};

// byte offsets of the device tables inside one allocation
struct PlanLayout {
    size_t desc, ftiles, fexec, btiles, bexec, gexec, fbegin, bbegin, fin, total;
};

namespace {
void trace_free(nurbs_plan* pl) {
    for (hipEvent_t e : pl->ev_f) (void)hipEventDestroy(e);
    for (hipEvent_t e : pl->ev_b) (void)hipEventDestroy(e);
    pl->ev_f.clear();
    pl->ev_b.clear();
    pl->trace_slots = 0;
    pl->calls_f = pl->calls_b = 0;
}
}  // namespace

namespace {

thread_local std::string g_noctx_err;

int fail(nurbs_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg; else g_noctx_err = msg;
    return code;
}

int hip_fail(nurbs_ctx* c, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, NURBS_EDEVICE, m);
}

int check_shape(nurbs_ctx* c, int p, int q, int nu_c, int nv_c, int nu_s, int nv_s) {
    if (p < 1 || q < 1 || p > NURBS_MAX_DEGREE || q > NURBS_MAX_DEGREE)
        return fail(c, NURBS_EDEGREE, "degree outside [1, " + std::to_string(NURBS_MAX_DEGREE) + "]");
    if (nu_c < p + 1 || nv_c < q + 1) return fail(c, NURBS_EDEGREE, "fewer control points than degree+1");
    if (nu_s < 0 || nv_s < 0) return fail(c, NURBS_EINVAL, "negative sample count");
    if ((long long)nu_c * nv_c > (1ll << 26)) return fail(c, NURBS_EINVAL, "control grid too large");
    static_assert(NURBS_MAX_KNOTS == kWG, "knot vectors are staged in kWG-entry LDS buffers");
    if (nu_c + p + 1 > NURBS_MAX_KNOTS || nv_c + q + 1 > NURBS_MAX_KNOTS)
        return fail(c, NURBS_EINVAL, "knot vector longer than " + std::to_string(NURBS_MAX_KNOTS));
    return NURBS_OK;
}

// Rows per tile from the surface's own shape only, so that a surface gets
// the same tiling -- and bitwise the same result -- alone, in a uniform
// batch or in any ragged mix.  A tile is one wave64 over min(64, nv_s)
// columns; the row count aims at a fixed number of points per tile.
int tile_rows(int nu_s, int nv_s, int target_pts) {
    const int cols = std::max(1, std::min(kWave, nv_s));
    const int rows = std::max(1, target_pts / cols);
    return std::max(1, std::min(std::max(nu_s, 1), rows));
}

}  // namespace

extern "C" {

const char* nurbs_status_string(int s) {
    switch (s) {
        case NURBS_OK: return "ok";
        case NURBS_EINVAL: return "invalid argument";
        case NURBS_EDEGREE: return "unsupported degree or too few control points";
        case NURBS_EKNOTS: return "invalid knot vector";
        case NURBS_EDOMAIN: return "sample outside the domain or unsorted";
        case NURBS_EWEIGHTS: return "non-positive weight";
        case NURBS_EWORKSPACE: return "workspace missing or too small";
        case NURBS_EDEVICE: return "HIP runtime error";
        case NURBS_EUNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

int nurbs_ctx_create(int device, nurbs_ctx** out) {
    if (!out) return fail(nullptr, NURBS_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(nullptr, NURBS_EINVAL, "no such device");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceProperties");
    nurbs_ctx* c = new nurbs_ctx();
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    *out = c;
    return NURBS_OK;
}

int nurbs_ctx_destroy(nurbs_ctx* ctx) {
    delete ctx;
    return NURBS_OK;
}

int nurbs_ctx_set_flags(nurbs_ctx* ctx, unsigned flags) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (flags & ~NURBS_VALIDATE) return fail(ctx, NURBS_EINVAL, "unknown flag bits");
    ctx->flags = flags;
    return NURBS_OK;
}

int nurbs_ctx_set_knot_sigma(nurbs_ctx* ctx, float sigma) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (sigma != 0.0f)
        return fail(ctx, NURBS_EUNSUPPORTED, "only the zero-bandwidth knot derivative (sigma = 0) is supported");
    return NURBS_OK;
}

int nurbs_ctx_set_tiling(nurbs_ctx* ctx, int fwd_tile_points, int bwd_tile_points) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    const int f = fwd_tile_points ? fwd_tile_points : 16384;
    const int b = bwd_tile_points ? bwd_tile_points : 16384;
    if (f < kWave || f > (1 << 22) || b < kWave || b > (1 << 22))
        return fail(ctx, NURBS_EINVAL, "tile points must be in [64, 4194304] (or 0 for the default)");
    ctx->fwd_tile_pts = f;
    ctx->bwd_tile_pts = b;
    return NURBS_OK;
}

int nurbs_ctx_set_schedule(nurbs_ctx* ctx, int schedule) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (schedule != NURBS_SCHED_STATIC && schedule != NURBS_SCHED_DYNAMIC)
        return fail(ctx, NURBS_EINVAL, "schedule must be NURBS_SCHED_STATIC or NURBS_SCHED_DYNAMIC");
    ctx->schedule = schedule;
    return NURBS_OK;
}

const char* nurbs_last_error(nurbs_ctx* ctx) { return ctx ? ctx->err.c_str() : g_noctx_err.c_str(); }

int nurbs_ctx_device_info(nurbs_ctx* ctx, int* num_cus, int* wave_size) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (num_cus) *num_cus = ctx->num_cus;
    if (wave_size) *wave_size = kWave;
    return NURBS_OK;
}

// --------------------------------------------------------------------------
// uniform batch
// --------------------------------------------------------------------------
namespace {

struct UniformGeom {
    int ncb, nrb_f, rows_f, nrb_b, rows_b;
    long long tiles_f, tiles_b;
    size_t slot;
};

UniformGeom uniform_geom(const nurbs_ctx* c, int B, int p, int q, int nu_c, int nv_c, int nu_s, int nv_s) {
    UniformGeom g;
    g.ncb = (nv_s + kWave - 1) / kWave;
    const long long cols = (long long)B * g.ncb;
    g.rows_f = tile_rows(nu_s, nv_s, c->fwd_tile_pts);
    g.rows_b = tile_rows(nu_s, nv_s, c->bwd_tile_pts);
    g.nrb_f = (nu_s + g.rows_f - 1) / g.rows_f;
    g.nrb_b = (nu_s + g.rows_b - 1) / g.rows_b;
    g.tiles_f = cols * g.nrb_f;
    g.tiles_b = cols * g.nrb_b;
    g.slot = slot_bytes(p, q, nu_c, nv_c, g.rows_b);
    return g;
}

constexpr size_t kWsHeader = 256;  // error word + padding
// plan workspaces: the 256-byte header, then the dynamic schedule's tile
// counters of the forward and of the backward (kQueues each, 128 bytes apart)
constexpr size_t kQueueFwd = kWsHeader;
constexpr size_t kQueueBwd = kQueueFwd + 4 * (size_t)kQueues * kQueueStride;
constexpr size_t kPlanHeader = kQueueBwd + 4 * (size_t)kQueues * kQueueStride;
static_assert(kPlanHeader == NURBS_PLAN_WS_HEADER, "plan workspace header");

int uniform_common(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, int nu_s, int nv_s) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (B < 0) return fail(ctx, NURBS_EINVAL, "negative batch");
    return check_shape(ctx, p, q, nu_c, nv_c, nu_s, nv_s);
}

UniformArgs make_uargs(const nurbs_ctx* ctx, const UniformGeom& g, bool bwd, int B, int nu_c, int nv_c,
                       int nu_s, int nv_s, const float* ctrl, const float* w, const float* ku,
                       const float* kv, const float* us, const float* vs, int uv_shared, void* ws) {
    UniformArgs a;
    a.ctrl = ctrl; a.w = w; a.ku = ku; a.kv = kv; a.us = us; a.vs = vs;
    a.B = B; a.nu_c = nu_c; a.nv_c = nv_c; a.nu_s = nu_s; a.nv_s = nv_s; a.uv_shared = uv_shared ? 1 : 0;
    a.ncb = g.ncb;
    a.nrb = bwd ? g.nrb_b : g.nrb_f;
    a.rows = bwd ? g.rows_b : g.rows_f;
    a.ntiles = (int)(bwd ? g.tiles_b : g.tiles_f);
    a.flags = ctx->flags;
    a.err = (ctx->flags & NURBS_VALIDATE) ? reinterpret_cast<int*>(ws) : nullptr;
    a.tab_u = a.tab_v = nullptr;
    a.tab_u_stride = a.tab_v_stride = 0;
    return a;
}

}  // namespace

int nurbs_surface_ws_bytes(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, int nu_s, int nv_s,
                           unsigned grad_mask, size_t* out) {
    int rc = uniform_common(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (rc) return rc;
    if (!out) return fail(ctx, NURBS_EINVAL, "out is NULL");
    if (grad_mask & ~NURBS_GRAD_ALL) return fail(ctx, NURBS_EINVAL, "unknown gradient bits");
    if (grad_mask == 0) {
        *out = (ctx->flags & NURBS_VALIDATE) ? kWsHeader : 0;
        return NURBS_OK;
    }
    const UniformGeom g = uniform_geom(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    *out = kWsHeader + (size_t)g.tiles_b * g.slot;
    return NURBS_OK;
}

int nurbs_surface_fwd(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, const float* ctrl,
                      const float* w, const float* ku, const float* kv, int nu_s, int nv_s, const float* us,
                      const float* vs, int uv_shared, float* pts, void* ws, size_t ws_bytes, void* stream) {
    int rc = uniform_common(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (rc) return rc;
    if (B == 0 || nu_s == 0 || nv_s == 0) return NURBS_OK;
    if (!ctrl || !w || !ku || !kv || !us || !vs || !pts) return fail(ctx, NURBS_EINVAL, "NULL array");
    if ((ctx->flags & NURBS_VALIDATE) && (!ws || ws_bytes < kWsHeader))
        return fail(ctx, NURBS_EWORKSPACE, "NURBS_VALIDATE needs a workspace");
    const UniformGeom g = uniform_geom(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (g.tiles_f > (1ll << 30)) return fail(ctx, NURBS_EINVAL, "batch too large");
    UniformArgs a = make_uargs(ctx, g, false, B, nu_c, nv_c, nu_s, nv_s, ctrl, w, ku, kv, us, vs, uv_shared, ws);
    const dim3 grid((unsigned)((g.tiles_f + kWavesPerWG - 1) / kWavesPerWG));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipErrorInvalidValue;
    switch (p) {
#define ND_CASE(P) case P: e = launch_uniform_fwd_p##P(q, grid, st, a, pts); break;
        ND_CASE(1) ND_CASE(2) ND_CASE(3) ND_CASE(4) ND_CASE(5) ND_CASE(6) ND_CASE(7)
#undef ND_CASE
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "launch forward");
    return NURBS_OK;
}

int nurbs_surface_derivs(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, const float* ctrl,
                         const float* w, const float* ku, const float* kv, int nu_s, int nv_s, const float* us,
                         const float* vs, int uv_shared, float* pts, float* pts_du, float* pts_dv, float* normals,
                         void* ws, size_t ws_bytes, void* stream) {
    int rc = uniform_common(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (rc) return rc;
    if (!pts && !pts_du && !pts_dv && !normals) return fail(ctx, NURBS_EINVAL, "no output requested");
    if (B == 0 || nu_s == 0 || nv_s == 0) return NURBS_OK;
    if (!ctrl || !w || !ku || !kv || !us || !vs) return fail(ctx, NURBS_EINVAL, "NULL array");
    if ((ctx->flags & NURBS_VALIDATE) && (!ws || ws_bytes < kWsHeader))
        return fail(ctx, NURBS_EWORKSPACE, "NURBS_VALIDATE needs a workspace");
    const UniformGeom g = uniform_geom(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (g.tiles_f > (1ll << 30)) return fail(ctx, NURBS_EINVAL, "batch too large");
    UniformArgs a = make_uargs(ctx, g, false, B, nu_c, nv_c, nu_s, nv_s, ctrl, w, ku, kv, us, vs, uv_shared, ws);
    const dim3 grid((unsigned)((g.tiles_f + kWavesPerWG - 1) / kWavesPerWG));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipErrorInvalidValue;
    switch (p) {
#define ND_CASE(P) case P: e = launch_uniform_der_p##P(q, grid, st, a, pts, pts_du, pts_dv, normals); break;
        ND_CASE(1) ND_CASE(2) ND_CASE(3) ND_CASE(4) ND_CASE(5) ND_CASE(6) ND_CASE(7)
#undef ND_CASE
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "launch derivatives");
    return NURBS_OK;
}

namespace {
// The gather of a uniform-batch backward: only dL/dP and dL/dw read the
// rectangles it writes.
hipError_t launch_uniform_gather(const nurbs_ctx* ctx, hipStream_t st, const UniformArgs& a, int p, int q,
                                 char* slots, size_t slot_sz, unsigned mask) {
    if (!(mask & (NURBS_GRAD_CTRL | NURBS_GRAD_W))) return hipSuccess;
    return q <= 5 ? launch_uniform_gat_d5(st, a, p, q, slots, slot_sz, ctx->num_cus)
                  : launch_uniform_gat_d7(st, a, p, q, slots, slot_sz, ctx->num_cus);
}
}  // namespace

int nurbs_surface_bwd(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, const float* ctrl,
                      const float* w, const float* ku, const float* kv, int nu_s, int nv_s, const float* us,
                      const float* vs, int uv_shared, const float* grad_pts, float* grad_ctrl, float* grad_w,
                      float* grad_ku, float* grad_kv, unsigned grad_mask, void* ws, size_t ws_bytes,
                      void* stream) {
    int rc = uniform_common(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (rc) return rc;
    if (grad_mask & ~NURBS_GRAD_ALL) return fail(ctx, NURBS_EINVAL, "unknown gradient bits");
    if (grad_mask == 0 || B == 0) return NURBS_OK;
    if (((grad_mask & NURBS_GRAD_CTRL) && !grad_ctrl) || ((grad_mask & NURBS_GRAD_W) && !grad_w) ||
        ((grad_mask & NURBS_GRAD_KU) && !grad_ku) || ((grad_mask & NURBS_GRAD_KV) && !grad_kv))
        return fail(ctx, NURBS_EINVAL, "NULL gradient output for a requested gradient");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (nu_s == 0 || nv_s == 0) {
        // no samples: every gradient is zero (no input is read, and empty
        // sample arrays may come as NULL)
        const size_t cp = (size_t)B * nu_c * nv_c;
        hipError_t e = hipSuccess;
        if (grad_mask & NURBS_GRAD_CTRL) e = launch_zero(st, grad_ctrl, cp * 3);
        if (!e && (grad_mask & NURBS_GRAD_W)) e = launch_zero(st, grad_w, cp);
        if (!e && (grad_mask & NURBS_GRAD_KU)) e = launch_zero(st, grad_ku, (size_t)B * (nu_c + p + 1));
        if (!e && (grad_mask & NURBS_GRAD_KV)) e = launch_zero(st, grad_kv, (size_t)B * (nv_c + q + 1));
        return e ? hip_fail(ctx, e, "zero fill") : NURBS_OK;
    }
    if (!ctrl || !w || !ku || !kv || !us || !vs) return fail(ctx, NURBS_EINVAL, "NULL array");
    if (!grad_pts) return fail(ctx, NURBS_EINVAL, "NULL grad_pts");
    const UniformGeom g = uniform_geom(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    const size_t need = kWsHeader + (size_t)g.tiles_b * g.slot;
    if (!ws || ws_bytes < need) return fail(ctx, NURBS_EWORKSPACE, "workspace too small: need " + std::to_string(need));
    if (g.tiles_b > (1ll << 30)) return fail(ctx, NURBS_EINVAL, "batch too large");
    const long long fin_items = (long long)B * fin_parts(nu_c, nv_c);
    if (fin_items > (1ll << 30)) return fail(ctx, NURBS_EINVAL, "batch too large");
    UniformArgs a = make_uargs(ctx, g, true, B, nu_c, nv_c, nu_s, nv_s, ctrl, w, ku, kv, us, vs, uv_shared, ws);
    char* slots = reinterpret_cast<char*>(ws) + kWsHeader;
    const dim3 grid((unsigned)((g.tiles_b + kWavesPerWG - 1) / kWavesPerWG));
    hipError_t e = hipErrorInvalidValue;
    switch (p) {
#define ND_CASE(P)                                                                                        \
    case P:                                                                                               \
        e = launch_uniform_bwd_p##P(q, grid, st, a, grad_pts, slots, g.slot, grad_mask);                  \
        if (e == hipSuccess) e = launch_uniform_gather(ctx, st, a, p, q, slots, g.slot, grad_mask);      \
        if (e == hipSuccess)                                                                              \
            e = launch_uniform_fin_p##P(q, dim3((fin_items + kWavesPerWG - 1) / kWavesPerWG), st, a, slots,  \
                                        g.slot,                                                           \
                                        grad_ctrl, grad_w, grad_ku,                                       \
                                        grad_kv, grad_mask);                                              \
        break;
        ND_CASE(1) ND_CASE(2) ND_CASE(3) ND_CASE(4) ND_CASE(5) ND_CASE(6) ND_CASE(7)
#undef ND_CASE
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "launch backward");
    return NURBS_OK;
}

// --------------------------------------------------------------------------
// fixed knots: precomputed span and basis tables
// --------------------------------------------------------------------------
namespace {
size_t table_bytes(int d, int n) { return basis_table_split(n) + sizeof(float) * (size_t)n * (d + 1); }
}  // namespace

int nurbs_basis_table_bytes(int p, int nx, size_t* out) {
    if (p < 1 || p > NURBS_MAX_DEGREE) return fail(nullptr, NURBS_EDEGREE, "degree");
    if (nx < 0 || !out) return fail(nullptr, NURBS_EINVAL, "bad arguments");
    *out = table_bytes(p, nx);
    return NURBS_OK;
}

int nurbs_basis_table_build(const float* knots, int n_knots, int p, const float* x, int nx, void* table,
                            size_t table_bytes_avail, void* stream) {
    if (p < 1 || p > NURBS_MAX_DEGREE) return fail(nullptr, NURBS_EDEGREE, "degree");
    if (n_knots < 2 * p + 2 || n_knots > NURBS_MAX_KNOTS || nx < 0 || !knots || (nx > 0 && (!x || !table)))
        return fail(nullptr, NURBS_EINVAL, "bad arguments");
    if (nx == 0) return NURBS_OK;
    if (table_bytes_avail < table_bytes(p, nx)) return fail(nullptr, NURBS_EWORKSPACE, "table too small");
    char* t = reinterpret_cast<char*>(table);
    hipError_t e = launch_spans(p, reinterpret_cast<hipStream_t>(stream), knots, n_knots, x, nx,
                                reinterpret_cast<int32_t*>(t), reinterpret_cast<float*>(t + basis_table_split(nx)));
    return e ? hip_fail(nullptr, e, "launch k_spans") : NURBS_OK;
}

namespace {
void bind_tables(UniformArgs& a, int p, int q, const void* tab_u, const void* tab_v, int tab_shared) {
    a.tab_u = reinterpret_cast<const char*>(tab_u);
    a.tab_v = reinterpret_cast<const char*>(tab_v);
    a.tab_u_stride = tab_shared ? 0 : table_bytes(p, a.nu_s);
    a.tab_v_stride = tab_shared ? 0 : table_bytes(q, a.nv_s);
}
}  // namespace

int nurbs_surface_fwd_tab(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, const float* ctrl,
                          const float* w, const float* ku, const float* kv, int nu_s, int nv_s, const float* us,
                          const float* vs, int uv_shared, const void* tab_u, const void* tab_v, int tab_shared,
                          float* pts, void* ws, size_t ws_bytes, void* stream) {
    int rc = uniform_common(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (rc) return rc;
    if (B == 0 || nu_s == 0 || nv_s == 0) return NURBS_OK;
    if (!ctrl || !w || !ku || !kv || !us || !vs || !pts || !tab_u || !tab_v)
        return fail(ctx, NURBS_EINVAL, "NULL array");
    if ((ctx->flags & NURBS_VALIDATE) && (!ws || ws_bytes < kWsHeader))
        return fail(ctx, NURBS_EWORKSPACE, "NURBS_VALIDATE needs a workspace");
    const UniformGeom g = uniform_geom(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (g.tiles_f > (1ll << 30)) return fail(ctx, NURBS_EINVAL, "batch too large");
    UniformArgs a = make_uargs(ctx, g, false, B, nu_c, nv_c, nu_s, nv_s, ctrl, w, ku, kv, us, vs, uv_shared, ws);
    bind_tables(a, p, q, tab_u, tab_v, tab_shared);
    const dim3 grid((unsigned)((g.tiles_f + kWavesPerWG - 1) / kWavesPerWG));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipErrorInvalidValue;
    switch (p) {
#define ND_CASE(P) case P: e = launch_uniform_fwd_p##P(q, grid, st, a, pts); break;
        ND_CASE(1) ND_CASE(2) ND_CASE(3) ND_CASE(4) ND_CASE(5) ND_CASE(6) ND_CASE(7)
#undef ND_CASE
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "launch forward (tables)");
    return NURBS_OK;
}

int nurbs_surface_bwd_tab(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, const float* ctrl,
                          const float* w, const float* ku, const float* kv, int nu_s, int nv_s, const float* us,
                          const float* vs, int uv_shared, const void* tab_u, const void* tab_v, int tab_shared,
                          const float* grad_pts, float* grad_ctrl, float* grad_w, unsigned grad_mask, void* ws,
                          size_t ws_bytes, void* stream) {
    int rc = uniform_common(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (rc) return rc;
    if (grad_mask & ~(NURBS_GRAD_CTRL | NURBS_GRAD_W))
        return fail(ctx, NURBS_EINVAL, "fixed knots: gradient bits are NURBS_GRAD_CTRL and NURBS_GRAD_W only");
    if (grad_mask == 0 || B == 0) return NURBS_OK;
    if (((grad_mask & NURBS_GRAD_CTRL) && !grad_ctrl) || ((grad_mask & NURBS_GRAD_W) && !grad_w))
        return fail(ctx, NURBS_EINVAL, "NULL gradient output for a requested gradient");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (nu_s == 0 || nv_s == 0) {  // no samples: zero gradients, no input read
        const size_t cp = (size_t)B * nu_c * nv_c;
        hipError_t e = hipSuccess;
        if (grad_mask & NURBS_GRAD_CTRL) e = launch_zero(st, grad_ctrl, cp * 3);
        if (!e && (grad_mask & NURBS_GRAD_W)) e = launch_zero(st, grad_w, cp);
        return e ? hip_fail(ctx, e, "zero fill") : NURBS_OK;
    }
    if (!ctrl || !w || !ku || !kv || !us || !vs) return fail(ctx, NURBS_EINVAL, "NULL array");
    if (!grad_pts || !tab_u || !tab_v) return fail(ctx, NURBS_EINVAL, "NULL grad_pts or table");
    const UniformGeom g = uniform_geom(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    const size_t need = kWsHeader + (size_t)g.tiles_b * g.slot;
    if (!ws || ws_bytes < need) return fail(ctx, NURBS_EWORKSPACE, "workspace too small: need " + std::to_string(need));
    if (g.tiles_b > (1ll << 30)) return fail(ctx, NURBS_EINVAL, "batch too large");
    const long long fin_items = (long long)B * fin_parts(nu_c, nv_c);
    if (fin_items > (1ll << 30)) return fail(ctx, NURBS_EINVAL, "batch too large");
    UniformArgs a = make_uargs(ctx, g, true, B, nu_c, nv_c, nu_s, nv_s, ctrl, w, ku, kv, us, vs, uv_shared, ws);
    bind_tables(a, p, q, tab_u, tab_v, tab_shared);
    char* slots = reinterpret_cast<char*>(ws) + kWsHeader;
    const dim3 grid((unsigned)((g.tiles_b + kWavesPerWG - 1) / kWavesPerWG));
    hipError_t e = hipErrorInvalidValue;
    switch (p) {
#define ND_CASE(P)                                                                                        \
    case P:                                                                                               \
        e = launch_uniform_bwd_p##P(q, grid, st, a, grad_pts, slots, g.slot, grad_mask);                  \
        if (e == hipSuccess) e = launch_uniform_gather(ctx, st, a, p, q, slots, g.slot, grad_mask);      \
        if (e == hipSuccess)                                                                              \
            e = launch_uniform_fin_p##P(q, dim3((fin_items + kWavesPerWG - 1) / kWavesPerWG), st, a, slots,  \
                                        g.slot, grad_ctrl, grad_w, nullptr, nullptr, grad_mask);          \
        break;
        ND_CASE(1) ND_CASE(2) ND_CASE(3) ND_CASE(4) ND_CASE(5) ND_CASE(6) ND_CASE(7)
#undef ND_CASE
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "launch backward (tables)");
    return NURBS_OK;
}

// --------------------------------------------------------------------------
// uniform backward without a caller workspace
// --------------------------------------------------------------------------
namespace {

// Device-resident scratch for nurbs_surface_bwd_noalloc: the backward's
// tile slots (and the 256-byte header) live here instead of in a caller
// workspace.  Every device the library runs on holds one copy until the
// process ends.  Host code must never pass `scratch` itself to a kernel
// (in host code it is a stand-in, not a device address): it uses the
// per-device address from hipGetSymbolAddress below.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The device address of this device's copy of `scratch`, looked up once per
// device with that device current.
int scratch_address(nurbs_ctx* ctx, void** out) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(ctx, NURBS_EINVAL, "device ordinal too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[ctx->device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipGetDevice");
        if (cur != ctx->device) return fail(ctx, NURBS_EINVAL, "the context's device is not the current device");
        void* addr = nullptr;
        e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(ctx, e, "hipGetSymbolAddress(scratch)");
        if (!addr) return fail(ctx, NURBS_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_addr[ctx->device] = addr;
    }
    *out = g_scratch_addr[ctx->device];
    return NURBS_OK;
}

}  // namespace

int nurbs_surface_bwd_noalloc(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, const float* ctrl,
                              const float* w, const float* ku, const float* kv, int nu_s, int nv_s, const float* us,
                              const float* vs, int uv_shared, const float* grad_pts, float* grad_ctrl, float* grad_w,
                              float* grad_ku, float* grad_kv, unsigned grad_mask, void* stream) {
    int rc = uniform_common(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s);
    if (rc) return rc;
    if (ctx->flags & NURBS_VALIDATE)
        return fail(ctx, NURBS_EUNSUPPORTED,
                    "nurbs_surface_bwd_noalloc runs no device-side data checks; clear NURBS_VALIDATE");
    if (grad_mask & ~NURBS_GRAD_ALL) return fail(ctx, NURBS_EINVAL, "unknown gradient bits");
    size_t need = 0;
    rc = nurbs_surface_ws_bytes(ctx, B, p, q, nu_c, nv_c, nu_s, nv_s, grad_mask, &need);
    if (rc) return rc;
    if (need > kNoAllocScratchBytes)
        return fail(ctx, NURBS_EWORKSPACE,
                    "this backward needs " + std::to_string(need) + " bytes of scratch; the built-in scratch holds " +
                        std::to_string(kNoAllocScratchBytes) + " (use nurbs_surface_bwd with a workspace)");
    void* ws = nullptr;
    rc = scratch_address(ctx, &ws);
    if (rc) return rc;
    // same kernels as nurbs_surface_bwd; every slot the finalize reads is
    // written by the backward kernel of the same call, and no error word is
    // used (NURBS_VALIDATE is refused), so nothing needs clearing first
    return nurbs_surface_bwd(ctx, B, p, q, nu_c, nv_c, ctrl, w, ku, kv, nu_s, nv_s, us, vs, uv_shared, grad_pts,
                             grad_ctrl, grad_w, grad_ku, grad_kv, grad_mask, ws, kNoAllocScratchBytes, stream);
}

// --------------------------------------------------------------------------
// curves
// --------------------------------------------------------------------------
namespace {

int curve_common(nurbs_ctx* ctx, int B, int p, int nc, int dim, int ns) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (B < 0 || ns < 0) return fail(ctx, NURBS_EINVAL, "negative batch or sample count");
    if (dim != 2 && dim != 3) return fail(ctx, NURBS_EINVAL, "dim must be 2 or 3");
    if (p < 1 || p > NURBS_MAX_DEGREE)
        return fail(ctx, NURBS_EDEGREE, "degree outside [1, " + std::to_string(NURBS_MAX_DEGREE) + "]");
    if (nc < p + 1) return fail(ctx, NURBS_EDEGREE, "fewer control points than degree+1");
    if (nc + p + 1 > NURBS_MAX_KNOTS)
        return fail(ctx, NURBS_EINVAL, "knot vector longer than " + std::to_string(NURBS_MAX_KNOTS));
    return NURBS_OK;
}

CurveArgs curve_args(const nurbs_ctx* ctx, int B, int p, int nc, int ns, const float* ctrl, const float* w,
                     const float* knots, const float* us, int u_shared, void* ws) {
    CurveArgs a;
    a.ctrl = ctrl; a.w = w; a.knots = knots; a.us = us;
    a.B = B; a.nc = nc; a.ns = ns; a.u_shared = u_shared ? 1 : 0;
    a.nchunks = std::max(1, (ns + kCurveChunk - 1) / kCurveChunk);
    a.part_floats = (4 * nc + nc + p + 1 + 3) & ~3;
    a.err = (ctx->flags & NURBS_VALIDATE) ? reinterpret_cast<int*>(ws) : nullptr;
    return a;
}

size_t curve_ws_need(const CurveArgs& a, bool bwd) {
    size_t n = (a.err || bwd) ? kWsHeader : 0;
    if (bwd && a.nchunks > 1) n += (size_t)a.B * a.nchunks * a.part_floats * sizeof(float);
    return n;
}

}  // namespace

int nurbs_curve_ws_bytes(nurbs_ctx* ctx, int B, int p, int nc, int dim, int ns, unsigned grad_mask, size_t* out) {
    int rc = curve_common(ctx, B, p, nc, dim, ns);
    if (rc) return rc;
    if (!out) return fail(ctx, NURBS_EINVAL, "out is NULL");
    if (grad_mask & ~(NURBS_GRAD_CTRL | NURBS_GRAD_W | NURBS_GRAD_KU))
        return fail(ctx, NURBS_EINVAL, "curve gradient bits are CTRL, W and KU (the knots)");
    const CurveArgs a = curve_args(ctx, B, p, nc, ns, nullptr, nullptr, nullptr, nullptr, 0, nullptr);
    if (grad_mask == 0) *out = (ctx->flags & NURBS_VALIDATE) ? kWsHeader : 0;
    else *out = curve_ws_need(a, true);
    return NURBS_OK;
}

int nurbs_curve_fwd(nurbs_ctx* ctx, int B, int p, int nc, int dim, const float* ctrl, const float* w,
                    const float* knots, int ns, const float* us, int u_shared, float* pts, float* pts_du, void* ws,
                    size_t ws_bytes, void* stream) {
    int rc = curve_common(ctx, B, p, nc, dim, ns);
    if (rc) return rc;
    if (B == 0 || ns == 0) return NURBS_OK;
    if (!ctrl || !w || !knots || !us || !pts) return fail(ctx, NURBS_EINVAL, "NULL array");
    if ((ctx->flags & NURBS_VALIDATE) && (!ws || ws_bytes < kWsHeader))
        return fail(ctx, NURBS_EWORKSPACE, "NURBS_VALIDATE needs a workspace");
    const CurveArgs a = curve_args(ctx, B, p, nc, ns, ctrl, w, knots, us, u_shared, ws);
    if ((long long)B * a.nchunks > (1ll << 31) - 1) return fail(ctx, NURBS_EINVAL, "batch too large");
    hipError_t e = launch_curve_fwd(p, dim, reinterpret_cast<hipStream_t>(stream), a, pts, pts_du);
    return e ? hip_fail(ctx, e, "launch curve forward") : NURBS_OK;
}

int nurbs_curve_bwd(nurbs_ctx* ctx, int B, int p, int nc, int dim, const float* ctrl, const float* w,
                    const float* knots, int ns, const float* us, int u_shared, const float* grad_pts,
                    float* grad_ctrl, float* grad_w, float* grad_knots, unsigned grad_mask, void* ws,
                    size_t ws_bytes, void* stream) {
    int rc = curve_common(ctx, B, p, nc, dim, ns);
    if (rc) return rc;
    if (grad_mask & ~(NURBS_GRAD_CTRL | NURBS_GRAD_W | NURBS_GRAD_KU))
        return fail(ctx, NURBS_EINVAL, "curve gradient bits are CTRL, W and KU (the knots)");
    if (grad_mask == 0 || B == 0) return NURBS_OK;
    if (((grad_mask & NURBS_GRAD_CTRL) && !grad_ctrl) || ((grad_mask & NURBS_GRAD_W) && !grad_w) ||
        ((grad_mask & NURBS_GRAD_KU) && !grad_knots))
        return fail(ctx, NURBS_EINVAL, "NULL gradient output for a requested gradient");
    if (!ctrl || !w || !knots) return fail(ctx, NURBS_EINVAL, "NULL array");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (ns == 0) {
        hipError_t e = hipSuccess;
        if (grad_mask & NURBS_GRAD_CTRL) e = launch_zero(st, grad_ctrl, (size_t)B * nc * dim);
        if (!e && (grad_mask & NURBS_GRAD_W)) e = launch_zero(st, grad_w, (size_t)B * nc);
        if (!e && (grad_mask & NURBS_GRAD_KU)) e = launch_zero(st, grad_knots, (size_t)B * (nc + p + 1));
        return e ? hip_fail(ctx, e, "zero fill") : NURBS_OK;
    }
    if (!us || !grad_pts) return fail(ctx, NURBS_EINVAL, "NULL us or grad_pts");
    const CurveArgs a = curve_args(ctx, B, p, nc, ns, ctrl, w, knots, us, u_shared, ws);
    const size_t need = curve_ws_need(a, true);
    if (!ws || ws_bytes < need) return fail(ctx, NURBS_EWORKSPACE, "workspace too small: need " + std::to_string(need));
    if ((long long)B * a.nchunks > (1ll << 31) - 1) return fail(ctx, NURBS_EINVAL, "batch too large");
    float* part = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + kWsHeader);
    hipError_t e = launch_curve_bwd(p, dim, st, a, grad_pts, grad_ctrl, grad_w, grad_knots, part, grad_mask);
    return e ? hip_fail(ctx, e, "launch curve backward") : NURBS_OK;
}

// --------------------------------------------------------------------------
// surfaces at scattered (u, v) pairs
// --------------------------------------------------------------------------
namespace {

struct UvLayout {
    size_t maxbits, acc, total;
};

UvLayout uv_layout(int B, int p, int q, int nu_c, int nv_c) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t nacc = 4 * (size_t)nu_c * nv_c + (nu_c + p + 1) + (nv_c + q + 1);
    UvLayout l;
    l.maxbits = kWsHeader;
    l.acc = l.maxbits + al(sizeof(unsigned) * 4 * (size_t)B);
    l.total = l.acc + al(sizeof(unsigned long long) * nacc * (size_t)B);
    return l;
}

int uv_common(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, int npts) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (B < 0 || npts < 0) return fail(ctx, NURBS_EINVAL, "negative batch or pair count");
    if (B > 65535) return fail(ctx, NURBS_EINVAL, "batch too large");
    return check_shape(ctx, p, q, nu_c, nv_c, npts, 1);
}

UvArgs uv_args(const nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, int npts, const float* ctrl,
               const float* w, const float* ku, const float* kv, const float* uv, int uv_shared, void* ws) {
    UvArgs a;
    a.ctrl = ctrl; a.w = w; a.ku = ku; a.kv = kv; a.uv = uv;
    a.B = B; a.p = p; a.q = q; a.nu_c = nu_c; a.nv_c = nv_c; a.npts = npts; a.uv_shared = uv_shared ? 1 : 0;
    a.nacc = 4 * nu_c * nv_c + (nu_c + p + 1) + (nv_c + q + 1);
    a.lds_acc = a.nacc <= kUvLdsAccMax ? 1 : 0;
    // pairs per backward workgroup: about 2048 workgroups over the batch;
    // with LDS accumulators at least 1024 pairs, so that the one flush of a
    // workgroup's accumulators stays small against its pairs
    const long long total = (long long)B * npts;
    long long c = ((total + 2047) / 2048 + 255) / 256 * 256;
    c = std::max<long long>(c, a.lds_acc ? 1024 : 256);
    a.chunk = (int)std::min<long long>(c, 16384);
    const size_t acc_lds = a.lds_acc ? 8 * (size_t)((a.nacc + 1) & ~1) : 0;
    a.lds_net = acc_lds + 16 * (size_t)nu_c * nv_c <= kUvLdsDynMax ? 1 : 0;
    // forward: 1024 pairs per workgroup when the net is staged (the staging
    // is shared by more pairs), else 256
    a.fchunk = a.lds_net ? 1024 : 256;
    a.err = (ctx->flags & NURBS_VALIDATE) ? reinterpret_cast<int*>(ws) : nullptr;
    return a;
}

}  // namespace

int nurbs_surface_uv_ws_bytes(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, int npts, unsigned grad_mask,
                              size_t* out) {
    int rc = uv_common(ctx, B, p, q, nu_c, nv_c, npts);
    if (rc) return rc;
    if (!out) return fail(ctx, NURBS_EINVAL, "out is NULL");
    if (grad_mask & ~NURBS_GRAD_ALL) return fail(ctx, NURBS_EINVAL, "unknown gradient bits");
    if (grad_mask == 0) *out = (ctx->flags & NURBS_VALIDATE) ? kWsHeader : 0;
    else *out = uv_layout(B, p, q, nu_c, nv_c).total;
    return NURBS_OK;
}

int nurbs_surface_uv_fwd(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, const float* ctrl, const float* w,
                         const float* ku, const float* kv, int npts, const float* uv, int uv_shared, float* pts,
                         float* pts_du, float* pts_dv, void* ws, size_t ws_bytes, void* stream) {
    int rc = uv_common(ctx, B, p, q, nu_c, nv_c, npts);
    if (rc) return rc;
    if (!pts && !pts_du && !pts_dv) return fail(ctx, NURBS_EINVAL, "no output requested");
    if (B == 0 || npts == 0) return NURBS_OK;
    if (!ctrl || !w || !ku || !kv || !uv) return fail(ctx, NURBS_EINVAL, "NULL array");
    if ((ctx->flags & NURBS_VALIDATE) && (!ws || ws_bytes < kWsHeader))
        return fail(ctx, NURBS_EWORKSPACE, "NURBS_VALIDATE needs a workspace");
    const UvArgs a = uv_args(ctx, B, p, q, nu_c, nv_c, npts, ctrl, w, ku, kv, uv, uv_shared, ws);
    hipError_t e = launch_uv_fwd(a, reinterpret_cast<hipStream_t>(stream), pts, pts_du, pts_dv);
    return e ? hip_fail(ctx, e, "launch uv forward") : NURBS_OK;
}

int nurbs_surface_uv_bwd(nurbs_ctx* ctx, int B, int p, int q, int nu_c, int nv_c, const float* ctrl, const float* w,
                         const float* ku, const float* kv, int npts, const float* uv, int uv_shared,
                         const float* grad_pts, float* grad_ctrl, float* grad_w, float* grad_ku, float* grad_kv,
                         unsigned grad_mask, void* ws, size_t ws_bytes, void* stream) {
    int rc = uv_common(ctx, B, p, q, nu_c, nv_c, npts);
    if (rc) return rc;
    if (grad_mask & ~NURBS_GRAD_ALL) return fail(ctx, NURBS_EINVAL, "unknown gradient bits");
    if (grad_mask == 0 || B == 0) return NURBS_OK;
    if (((grad_mask & NURBS_GRAD_CTRL) && !grad_ctrl) || ((grad_mask & NURBS_GRAD_W) && !grad_w) ||
        ((grad_mask & NURBS_GRAD_KU) && !grad_ku) || ((grad_mask & NURBS_GRAD_KV) && !grad_kv))
        return fail(ctx, NURBS_EINVAL, "NULL gradient output for a requested gradient");
    if (!ctrl || !w || !ku || !kv) return fail(ctx, NURBS_EINVAL, "NULL array");
    const UvLayout l = uv_layout(B, p, q, nu_c, nv_c);
    if (!ws || ws_bytes < l.total) return fail(ctx, NURBS_EWORKSPACE, "workspace too small: need " + std::to_string(l.total));
    if (npts > 0 && (!uv || !grad_pts)) return fail(ctx, NURBS_EINVAL, "NULL uv or grad_pts");
    const UvArgs a = uv_args(ctx, B, p, q, nu_c, nv_c, npts, ctrl, w, ku, kv, uv, uv_shared, ws);
    char* wb = reinterpret_cast<char*>(ws);
    hipError_t e = launch_uv_bwd(a, reinterpret_cast<hipStream_t>(stream), grad_pts, grad_mask,
                                 reinterpret_cast<unsigned*>(wb + l.maxbits),
                                 reinterpret_cast<unsigned long long*>(wb + l.acc), grad_ctrl, grad_w, grad_ku, grad_kv);
    return e ? hip_fail(ctx, e, "launch uv backward") : NURBS_OK;
}

// --------------------------------------------------------------------------
// point-set losses
// --------------------------------------------------------------------------
namespace {

struct CdLayout {
    size_t a, da, b, db, state, part, acc, pidx, pd2, total;
};

// Workspace of nurbs_nearest / nurbs_chamfer: the 256-byte header, both
// nearest-neighbour maps, the per-pair state and the per-range partials of
// the larger of the two searches.
CdLayout cd_layout(int B, int n, int m, int num_cus) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const NnSplit s1 = nn_split(B, n, m, num_cus), s2 = nn_split(B, m, n, num_cus);
    const size_t part = std::max(s1.nranges > 1 ? (size_t)s1.nranges * n : 0, s2.nranges > 1 ? (size_t)s2.nranges * m : 0);
    CdLayout l;
    l.a = kWsHeader;
    l.da = l.a + al(sizeof(int) * (size_t)B * n);
    l.b = l.da + al(sizeof(float) * (size_t)B * n);
    l.db = l.b + al(sizeof(int) * (size_t)B * m);
    l.state = l.db + al(sizeof(float) * (size_t)B * m);
    l.part = l.state + al(cd_state_bytes() * (size_t)B);
    l.acc = l.part + al(cd_part_bytes(n, m) * (size_t)B);
    l.pidx = l.acc + al(sizeof(unsigned long long) * 3 * (size_t)B * n);
    l.pd2 = l.pidx + al(sizeof(int) * (size_t)B * part);
    l.total = l.pd2 + al(sizeof(float) * (size_t)B * part);
    return l;
}

int cd_common(nurbs_ctx* ctx, int B, int dim, int n, int m) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (dim != 2 && dim != 3) return fail(ctx, NURBS_EINVAL, "dim must be 2 or 3");
    if (B < 0 || n < 1 || m < 1) return fail(ctx, NURBS_EINVAL, "need B >= 0 and at least one point in each set");
    if ((long long)B * n > (1ll << 30) || (long long)B * m > (1ll << 30) || B > 65535 || m > (1 << 22))
        return fail(ctx, NURBS_EINVAL, "point sets too large");
    return NURBS_OK;
}

}  // namespace

int nurbs_chamfer_ws_bytes(nurbs_ctx* ctx, int B, int n, int m, size_t* out) {
    int rc = cd_common(ctx, B, 3, n, m);
    if (rc) return rc;
    if (!out) return fail(ctx, NURBS_EINVAL, "out is NULL");
    *out = cd_layout(B, n, m, ctx->num_cus).total;
    return NURBS_OK;
}

int nurbs_nearest(nurbs_ctx* ctx, int B, int dim, const float* X, int n, const float* Y, int m, int32_t* idx,
                  float* d2, void* ws, size_t ws_bytes, void* stream) {
    int rc = cd_common(ctx, B, dim, n, m);
    if (rc) return rc;
    if (B == 0) return NURBS_OK;
    if (!X || !Y || !idx || !d2) return fail(ctx, NURBS_EINVAL, "NULL array");
    const CdLayout l = cd_layout(B, n, m, ctx->num_cus);
    const NnSplit sp = nn_split(B, n, m, ctx->num_cus);
    char* w = reinterpret_cast<char*>(ws);
    if (!ws || ws_bytes < l.total)
        return fail(ctx, NURBS_EWORKSPACE, "workspace too small: need " + std::to_string(l.total));
    hipError_t e = launch_nn(dim, reinterpret_cast<hipStream_t>(stream), B, X, n, Y, m, sp, idx, d2,
                             sp.nranges > 1 ? reinterpret_cast<int*>(w + l.pidx) : nullptr,
                             sp.nranges > 1 ? reinterpret_cast<float*>(w + l.pd2) : nullptr);
    return e ? hip_fail(ctx, e, "launch nearest") : NURBS_OK;
}

int nurbs_chamfer(nurbs_ctx* ctx, int B, int dim, const float* P, int n, const float* Q, int m, float* out,
                  float* grad_cd, float* grad_hd, void* ws, size_t ws_bytes, void* stream) {
    int rc = cd_common(ctx, B, dim, n, m);
    if (rc) return rc;
    if (B == 0) return NURBS_OK;
    if (!P || !Q || !out) return fail(ctx, NURBS_EINVAL, "NULL array");
    const CdLayout l = cd_layout(B, n, m, ctx->num_cus);
    if (!ws || ws_bytes < l.total) return fail(ctx, NURBS_EWORKSPACE, "workspace too small: need " + std::to_string(l.total));
    char* w = reinterpret_cast<char*>(ws);
    int* a = reinterpret_cast<int*>(w + l.a);
    float* da = reinterpret_cast<float*>(w + l.da);
    int* bq = reinterpret_cast<int*>(w + l.b);
    float* db = reinterpret_cast<float*>(w + l.db);
    int* pidx = reinterpret_cast<int*>(w + l.pidx);
    float* pd2 = reinterpret_cast<float*>(w + l.pd2);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_nn(dim, st, B, P, n, Q, m, nn_split(B, n, m, ctx->num_cus), a, da, pidx, pd2);
    if (e == hipSuccess) e = launch_nn(dim, st, B, Q, m, P, n, nn_split(B, m, n, ctx->num_cus), bq, db, pidx, pd2);
    if (e == hipSuccess)
        e = launch_cd(dim, st, B, P, n, Q, m, a, da, bq, db, out, w + l.state, w + l.part, w + l.acc, grad_cd, grad_hd);
    return e ? hip_fail(ctx, e, "launch chamfer") : NURBS_OK;
}

// --------------------------------------------------------------------------
// plans
// --------------------------------------------------------------------------
namespace {

// Estimated wave time of a tile (arbitrary units, about a microsecond): a
// fixed set-up (dependent loads of the tile's tables, knots and first
// control rows), a per-row cost growing with the degree in u and, in the
// backward, a per-control-row flush growing with the degree in v.
double tile_cost(const nurbs_desc& d, int rows, bool bwd) {
    if (!bwd) return 9.0 + rows * (0.40 + 0.06 * (d.p + 1));
    const double crow = std::min<double>(d.nu_c, d.p + 1 + (double)rows * (d.nu_c - d.p) / std::max(d.nu_s, 1));
    return 12.0 + rows * (1.0 + 0.25 * (d.p + 1)) + crow * (0.5 + 0.35 * (d.q + 1));
}

// Estimated work of a backward tile's gather: its blocks of four control rows
// by 16 control columns (the expected rows and columns the tile touches).
double gather_cost(const nurbs_desc& d, int rows, int cols) {
    const double crow = std::min<double>(d.nu_c, d.p + 1 + (double)rows * (d.nu_c - d.p) / std::max(d.nu_s, 1));
    const double ccol = std::min<double>(d.nv_c, d.q + 1 + (double)cols * (d.nv_c - d.q) / std::max(d.nv_s, 1));
    return std::ceil(crow / 4.0) * std::ceil(ccol / 16.0);
}

// Tiles by decreasing estimated cost (ties in tile order).
std::vector<int> longest_first(const std::vector<double>& cost) {
    std::vector<int> idx(cost.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    return idx;
}

// Static schedule: assign tiles to nw waves, longest first, each to the wave
// with the least work so far.  Returns the tiles in wave order and the wave
// boundaries.  Dynamic schedule: the longest-first order itself (the waves
// take tiles from it at run time); the boundaries are unused.
void assign_waves(const std::vector<double>& cost, int nw, std::vector<int>& order, std::vector<int>& begin,
                  bool dynamic) {
    std::vector<int> idx = longest_first(cost);
    if (dynamic) {
        order = idx;
        begin.assign(nw + 1, 0);
        return;
    }
    using Load = std::pair<double, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int w = 0; w < nw; ++w) heap.push({0.0, w});
    std::vector<std::vector<int>> lists(nw);
    for (int t : idx) {
        Load l = heap.top();
        heap.pop();
        lists[l.second].push_back(t);
        l.first += cost[t];
        heap.push(l);
    }
    order.clear();
    begin.assign(nw + 1, 0);
    for (int w = 0; w < nw; ++w) {
        begin[w] = (int)order.size();
        order.insert(order.end(), lists[w].begin(), lists[w].end());
    }
    begin[nw] = (int)order.size();
}

}  // namespace

namespace {
// Host half of plan creation: validate the descriptors, cut tiles, assign
// them to waves and lay out the device tables in *blob.  The device pointers
// are bound by plan_bind once the blob has a device address.  With blob ==
// NULL only the sizes (layout, workspace) are worked out.
int plan_build(nurbs_ctx* ctx, const nurbs_desc* host, int n, unsigned flags, nurbs_plan** out,
               std::vector<char>* blob, PlanLayout* lay) {
    if (!ctx) return fail(nullptr, NURBS_EINVAL, "ctx is NULL");
    if (!out || (!host && n > 0) || n < 0) return fail(ctx, NURBS_EINVAL, "bad arguments");
    if (flags & ~NURBS_VALIDATE) return fail(ctx, NURBS_EINVAL, "unknown flag bits");
    *out = nullptr;
    for (int s = 0; s < n; ++s) {
        const nurbs_desc& d = host[s];
        int rc = check_shape(ctx, d.p, d.q, d.nu_c, d.nv_c, d.nu_s, d.nv_s);
        if (rc) {
            ctx->err = "surface " + std::to_string(s) + ": " + ctx->err;
            return rc;
        }
        if (d.ctrl_off < 0 || d.w_off < 0 || d.ku_off < 0 || d.kv_off < 0 || d.us_off < 0 || d.vs_off < 0 ||
            d.pts_off < 0)
            return fail(ctx, NURBS_EINVAL, "surface " + std::to_string(s) + ": negative offset");
    }
    nurbs_plan* pl = new nurbs_plan();
    pl->ctx = ctx;
    pl->device = ctx->device;
    pl->n = n;
    pl->flags = flags;
    pl->schedule = ctx->schedule;
    pl->host.assign(host, host + n);

    // tiles
    std::vector<DevDesc> dd(n);
    std::vector<DevTile> ft, bt;
    std::vector<double> fcost, bcost, gcost;
    size_t slot_off = 0;
    const int cus = std::max(ctx->num_cus, 1);
    for (int s = 0; s < n; ++s) {
        const nurbs_desc& d = pl->host[s];
        DevDesc& x = dd[s];
        x.p = d.p; x.q = d.q; x.nu_c = d.nu_c; x.nv_c = d.nv_c; x.nu_s = d.nu_s; x.nv_s = d.nv_s;
        x.ctrl_off = d.ctrl_off; x.w_off = d.w_off; x.ku_off = d.ku_off; x.kv_off = d.kv_off;
        x.us_off = d.us_off; x.vs_off = d.vs_off; x.pts_off = d.pts_off;
        x.pad = 0;
        const int ncb = (d.nv_s + kWave - 1) / kWave;
        const int rf = tile_rows(d.nu_s, d.nv_s, ctx->fwd_tile_pts);
        const int rb = tile_rows(d.nu_s, d.nv_s, ctx->bwd_tile_pts);
        x.rows = rb;
        x.tile_first = (int)bt.size();
        x.slot0 = (long long)(kPlanHeader + slot_off);
        int cnt = 0;
        if (d.nu_s > 0 && d.nv_s > 0) {
            for (int r0 = 0; r0 < d.nu_s; r0 += rf)
                for (int cb = 0; cb < ncb; ++cb) {
                    DevTile t{s, cb * kWave, r0, std::min(d.nu_s, r0 + rf), 0};
                    ft.push_back(t);
                    fcost.push_back(tile_cost(d, t.row1 - t.row0, false));
                }
            for (int r0 = 0; r0 < d.nu_s; r0 += rb)
                for (int cb = 0; cb < ncb; ++cb) {
                    DevTile t{s, cb * kWave, r0, std::min(d.nu_s, r0 + rb), (long long)(kPlanHeader + slot_off)};
                    slot_off += align16(slot_bytes(d.p, d.q, d.nu_c, d.nv_c, rb));
                    bt.push_back(t);
                    bcost.push_back(tile_cost(d, t.row1 - t.row0, true));
                    gcost.push_back(gather_cost(d, t.row1 - t.row0, std::min(kWave, d.nv_s - t.col0)));
                    ++cnt;
                }
        }
        x.tile_count = cnt;
        pl->max_nU = std::max(pl->max_nU, d.nu_c + d.p + 1);
        pl->max_nV = std::max(pl->max_nV, d.nv_c + d.q + 1);
    }
    pl->nf = (int)ft.size();
    pl->nb = (int)bt.size();
    pl->ws_bytes = kPlanHeader + slot_off;

    // degree class and persistent grid: as many workgroups as fit at once
    int maxdeg = 1;
    for (const auto& d : pl->host) maxdeg = std::max(maxdeg, std::max(d.p, d.q));
    pl->maxd = maxdeg <= 5 ? 5 : 7;
    int* occ = ctx->occ[pl->maxd == 5 ? 0 : 1];
    if (occ[0] == 0 || occ[1] == 0) {  // asked once per context
        hipError_t e = pl->maxd == 5 ? occupancy_plan_fwd_d5(&occ[0]) : occupancy_plan_fwd_d7(&occ[0]);
        if (e == hipSuccess) e = pl->maxd == 5 ? occupancy_plan_bwd_d5(&occ[1]) : occupancy_plan_bwd_d7(&occ[1]);
        if (e != hipSuccess) {
            occ[0] = occ[1] = 0;
            delete pl;
            return hip_fail(ctx, e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
        }
    }
    const int occ_f = std::max(occ[0], 1), occ_b = std::max(occ[1], 1);
    pl->grid_fwd = std::max(1, std::min(occ_f * cus, (pl->nf + kWavesPerWG - 1) / kWavesPerWG));
    pl->grid_bwd = std::max(1, std::min(occ_b * cus, (pl->nb + kWavesPerWG - 1) / kWavesPerWG));
    // finalize parts, most expensive first (estimated dependent memory rounds)
    std::vector<int2> fin;
    std::vector<double> fin_cost;
    for (int s = 0; s < n; ++s) {
        const nurbs_desc& d = pl->host[s];
        const int ncb = (d.nv_s + kWave - 1) / kWave;
        const int nrb = dd[s].tile_count > 0 && ncb > 0 ? dd[s].tile_count / ncb : 0;
        const int np = fin_parts(d.nu_c, d.nv_c);
        for (int part = 0; part < np; ++part) {
            double c;
            if (part == kFinKU) c = 4.0 + ((d.nu_s + kWave - 1) / kWave) * (2.0 + ncb + 0.2 * (d.p + 1));
            else if (part == kFinKV) c = 4.0 + ((d.nv_s + kWave - 1) / kWave) * (2.0 + nrb + 0.2 * (d.q + 1));
            else c = 3.0 + dd[s].tile_count;
            fin.push_back(make_int2(s, part));
            fin_cost.push_back(c);
        }
    }
    {
        std::vector<int> idx(fin.size());
        std::iota(idx.begin(), idx.end(), 0);
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return fin_cost[x] > fin_cost[y]; });
        std::vector<int2> sorted(fin.size());
        for (size_t i = 0; i < idx.size(); ++i) sorted[i] = fin[idx[i]];
        fin.swap(sorted);
    }
    pl->nfin = (int)fin.size();

    // table layout (sizes follow from the counts alone)
    const size_t nwf = (size_t)pl->grid_fwd * kWavesPerWG, nwb = (size_t)pl->grid_bwd * kWavesPerWG;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_desc = 0;
    const size_t o_ft = o_desc + al(sizeof(DevDesc) * std::max(n, 1));
    const size_t o_fx = o_ft + al(sizeof(DevTile) * std::max<size_t>(ft.size(), 1));
    const size_t o_bt = o_fx + al(sizeof(ExecTile) * std::max<size_t>(ft.size(), 1));
    const size_t o_bx = o_bt + al(sizeof(DevTile) * std::max<size_t>(bt.size(), 1));
    const size_t o_gx = o_bx + al(sizeof(ExecTile) * std::max<size_t>(bt.size(), 1));
    const size_t o_fb = o_gx + al(sizeof(ExecTile) * std::max<size_t>(bt.size(), 1));
    const size_t o_bb = o_fb + al(sizeof(int) * (nwf + 1));
    const size_t o_fi = o_bb + al(sizeof(int) * (nwb + 1));
    const size_t total = o_fi + al(sizeof(int2) * std::max<size_t>(fin.size(), 1));
    if (!blob) {  // size query: no schedule, no tables
        *lay = PlanLayout{o_desc, o_ft, o_fx, o_bt, o_bx, o_gx, o_fb, o_bb, o_fi, total};
        *out = pl;
        return NURBS_OK;
    }
    std::vector<int> fo, fbeg, bo, bbeg;
    assign_waves(fcost, (int)nwf, fo, fbeg, pl->schedule == NURBS_SCHED_DYNAMIC);
    assign_waves(bcost, (int)nwb, bo, bbeg, pl->schedule == NURBS_SCHED_DYNAMIC);
    auto record = [&](const DevTile& t) {
        const DevDesc& x = dd[t.surf];
        ExecTile r;
        r.p = x.p; r.q = x.q; r.nu_c = x.nu_c; r.nv_c = x.nv_c; r.nu_s = x.nu_s; r.nv_s = x.nv_s;
        r.col0 = t.col0; r.row0 = t.row0; r.row1 = t.row1; r.rows = x.rows;
        r.ctrl_off = x.ctrl_off; r.w_off = x.w_off; r.ku_off = x.ku_off; r.kv_off = x.kv_off;
        r.us_off = x.us_off; r.vs_off = x.vs_off; r.pts_off = x.pts_off; r.slot_off = t.slot_off;
        return r;
    };
    std::vector<ExecTile> fx, bx, gx;
    fx.reserve(fo.size());
    bx.reserve(bo.size());
    gx.reserve(bt.size());
    for (int i : fo) fx.push_back(record(ft[i]));
    for (int i : bo) bx.push_back(record(bt[i]));
    for (int i : longest_first(gcost)) gx.push_back(record(bt[i]));
    blob->assign(total, 0);
    char* hb = blob->data();
    if (n) memcpy(hb + o_desc, dd.data(), sizeof(DevDesc) * n);
    if (!ft.empty()) memcpy(hb + o_ft, ft.data(), sizeof(DevTile) * ft.size());
    if (!fx.empty()) memcpy(hb + o_fx, fx.data(), sizeof(ExecTile) * fx.size());
    if (!bt.empty()) memcpy(hb + o_bt, bt.data(), sizeof(DevTile) * bt.size());
    if (!bx.empty()) memcpy(hb + o_bx, bx.data(), sizeof(ExecTile) * bx.size());
    if (!gx.empty()) memcpy(hb + o_gx, gx.data(), sizeof(ExecTile) * gx.size());
    memcpy(hb + o_fb, fbeg.data(), sizeof(int) * fbeg.size());
    memcpy(hb + o_bb, bbeg.data(), sizeof(int) * bbeg.size());
    if (!fin.empty()) memcpy(hb + o_fi, fin.data(), sizeof(int2) * fin.size());
    *lay = PlanLayout{o_desc, o_ft, o_fx, o_bt, o_bx, o_gx, o_fb, o_bb, o_fi, total};
    *out = pl;
    return NURBS_OK;
}

void plan_bind(nurbs_plan* pl, void* dev, const PlanLayout& lay) {
    char* base = reinterpret_cast<char*>(dev);
    pl->d_desc = reinterpret_cast<DevDesc*>(base + lay.desc);
    pl->d_ftiles = reinterpret_cast<DevTile*>(base + lay.ftiles);
    pl->d_fexec = reinterpret_cast<ExecTile*>(base + lay.fexec);
    pl->d_btiles = reinterpret_cast<DevTile*>(base + lay.btiles);
    pl->d_bexec = reinterpret_cast<ExecTile*>(base + lay.bexec);
    pl->d_gexec = reinterpret_cast<ExecTile*>(base + lay.gexec);
    pl->d_fbegin = reinterpret_cast<int*>(base + lay.fbegin);
    pl->d_bbegin = reinterpret_cast<int*>(base + lay.bbegin);
    pl->d_fin = reinterpret_cast<int2*>(base + lay.fin);
}
}  // namespace

int nurbs_plan_create(nurbs_ctx* ctx, const nurbs_desc* host, int n, unsigned flags, nurbs_plan** out,
                      size_t* ws_bytes) {
    std::vector<char> blob;
    PlanLayout lay;
    nurbs_plan* pl = nullptr;
    int rc = plan_build(ctx, host, n, flags, &pl, &blob, &lay);
    if (rc) return rc;
    hipError_t e = hipMalloc(&pl->dev, lay.total);
    if (e != hipSuccess) {
        delete pl;
        return hip_fail(ctx, e, "hipMalloc(plan tables)");
    }
    e = hipMemcpy(pl->dev, blob.data(), lay.total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(pl->dev);
        delete pl;
        return hip_fail(ctx, e, "hipMemcpy(plan tables)");
    }
    plan_bind(pl, pl->dev, lay);
    *out = pl;
    if (ws_bytes) *ws_bytes = pl->ws_bytes;
    return NURBS_OK;
}

int nurbs_plan_create_in(nurbs_ctx* ctx, const nurbs_desc* host, int n, unsigned flags, void* tables,
                         size_t tables_bytes, void* stream, nurbs_plan** out, size_t* table_bytes_needed,
                         size_t* ws_bytes) {
    std::vector<char> blob;
    PlanLayout lay;
    nurbs_plan* pl = nullptr;
    if (out) *out = nullptr;
    nurbs_plan* tmp = nullptr;
    int rc = plan_build(ctx, host, n, flags, &tmp, tables ? &blob : nullptr, &lay);
    if (rc) return rc;
    pl = tmp;
    if (table_bytes_needed) *table_bytes_needed = lay.total;
    if (ws_bytes) *ws_bytes = pl->ws_bytes;
    if (!tables) {  // size query
        delete pl;
        return NURBS_OK;
    }
    if (!out) {
        delete pl;
        return fail(ctx, NURBS_EINVAL, "out is NULL");
    }
    if (tables_bytes < lay.total) {
        delete pl;
        return fail(ctx, NURBS_EWORKSPACE, "table memory too small: need " + std::to_string(lay.total));
    }
    // the blob stays with the plan until it is destroyed, so the asynchronous
    // copy never reads freed host memory
    pl->staging = std::move(blob);
    hipError_t e = hipMemcpyAsync(tables, pl->staging.data(), lay.total, hipMemcpyHostToDevice,
                                  reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        delete pl;
        return hip_fail(ctx, e, "hipMemcpyAsync(plan tables)");
    }
    plan_bind(pl, tables, lay);
    *out = pl;
    return NURBS_OK;
}

int nurbs_plan_destroy(nurbs_plan* plan) {
    if (!plan) return NURBS_OK;
    trace_free(plan);
    if (plan->dev) (void)hipFree(plan->dev);
    delete plan;
    return NURBS_OK;
}

int nurbs_plan_info(nurbs_plan* plan, int* fwd_tiles, int* bwd_tiles, int* grid) {
    if (!plan) return fail(nullptr, NURBS_EINVAL, "plan is NULL");
    if (fwd_tiles) *fwd_tiles = plan->nf;
    if (bwd_tiles) *bwd_tiles = plan->nb;
    if (grid) *grid = plan->grid_bwd;
    return NURBS_OK;
}

namespace {
PlanArgs plan_args(nurbs_plan* pl, bool bwd, void* ws, const float* ctrl, const float* w, const float* ku,
                   const float* kv, const float* us, const float* vs) {
    PlanArgs a;
    a.desc = pl->d_desc;
    a.tiles = bwd ? pl->d_btiles : pl->d_ftiles;
    a.exec = bwd ? pl->d_bexec : pl->d_fexec;
    a.gexec = bwd ? pl->d_gexec : nullptr;
    a.ntiles = bwd ? pl->nb : pl->nf;
    a.wave_begin = bwd ? pl->d_bbegin : pl->d_fbegin;
    a.nwaves = (bwd ? pl->grid_bwd : pl->grid_fwd) * kWavesPerWG;
    // dynamic schedule: the tile counters live in the workspace header
    a.queue = pl->schedule == NURBS_SCHED_DYNAMIC ? reinterpret_cast<int*>(reinterpret_cast<char*>(ws) +
                                                                             (bwd ? kQueueBwd : kQueueFwd))
                                                  : nullptr;
    a.flags = pl->flags;
    a.err = (pl->flags & NURBS_VALIDATE) ? reinterpret_cast<int*>(ws) : nullptr;
    a.ctrl = ctrl; a.w = w; a.ku = ku; a.kv = kv; a.us = us; a.vs = vs;
    a.nsurf = pl->n;
    a.fin_items = pl->d_fin;
    a.nfin = pl->nfin;
    return a;
}
}  // namespace

int nurbs_plan_fwd(nurbs_plan* pl, const float* ctrl, const float* w, const float* ku, const float* kv,
                   const float* us, const float* vs, float* pts, void* ws, size_t ws_bytes, void* stream) {
    if (!pl) return fail(nullptr, NURBS_EINVAL, "plan is NULL");
    if (pl->nf == 0) return NURBS_OK;
    if (!ctrl || !w || !ku || !kv || !us || !vs || !pts) return fail(pl->ctx, NURBS_EINVAL, "NULL array");
    if ((pl->flags & NURBS_VALIDATE) && (!ws || ws_bytes < kWsHeader))
        return fail(pl->ctx, NURBS_EWORKSPACE, "NURBS_VALIDATE needs a workspace");
    if (pl->schedule == NURBS_SCHED_DYNAMIC && (!ws || ws_bytes < kPlanHeader))
        return fail(pl->ctx, NURBS_EWORKSPACE, "the dynamic schedule needs the first NURBS_PLAN_WS_HEADER bytes of "
                                               "the plan's workspace");
    PlanArgs a = plan_args(pl, false, ws, ctrl, w, ku, kv, us, vs);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t* ev = nullptr;
    if (pl->trace_slots > 0) {
        ev = &pl->ev_f[2 * (size_t)(pl->calls_f % pl->trace_slots)];
        ++pl->calls_f;
        (void)hipEventRecord(ev[0], st);
    }
    hipError_t e = a.queue ? launch_zero(st, reinterpret_cast<float*>(a.queue), (size_t)kQueues * kQueueStride)
                           : hipSuccess;
    if (e == hipSuccess)
        e = pl->maxd == 5 ? launch_plan_fwd_d5(dim3(pl->grid_fwd), st, a, pts)
                          : launch_plan_fwd_d7(dim3(pl->grid_fwd), st, a, pts);
    if (ev && e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e != hipSuccess) return hip_fail(pl->ctx, e, "launch plan forward");
    return NURBS_OK;
}

int nurbs_plan_bwd(nurbs_plan* pl, const float* ctrl, const float* w, const float* ku, const float* kv,
                   const float* us, const float* vs, const float* grad_pts, float* grad_ctrl, float* grad_w,
                   float* grad_ku, float* grad_kv, unsigned grad_mask, void* ws, size_t ws_bytes, void* stream) {
    if (!pl) return fail(nullptr, NURBS_EINVAL, "plan is NULL");
    if (grad_mask & ~NURBS_GRAD_ALL) return fail(pl->ctx, NURBS_EINVAL, "unknown gradient bits");
    if (grad_mask == 0 || pl->n == 0) return NURBS_OK;
    if (((grad_mask & NURBS_GRAD_CTRL) && !grad_ctrl) || ((grad_mask & NURBS_GRAD_W) && !grad_w) ||
        ((grad_mask & NURBS_GRAD_KU) && !grad_ku) || ((grad_mask & NURBS_GRAD_KV) && !grad_kv))
        return fail(pl->ctx, NURBS_EINVAL, "NULL gradient output for a requested gradient");
    if (!ctrl || !w || !ku || !kv || !us || !vs || !grad_pts) return fail(pl->ctx, NURBS_EINVAL, "NULL array");
    if (!ws || ws_bytes < pl->ws_bytes)
        return fail(pl->ctx, NURBS_EWORKSPACE, "workspace too small: need " + std::to_string(pl->ws_bytes));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PlanArgs a = plan_args(pl, true, ws, ctrl, w, ku, kv, us, vs);
    char* slots = reinterpret_cast<char*>(ws);
    hipError_t e = hipSuccess;
    hipEvent_t* ev = nullptr;
    if (pl->trace_slots > 0) {
        ev = &pl->ev_b[4 * (size_t)(pl->calls_b % pl->trace_slots)];
        ++pl->calls_b;
        e = hipEventRecord(ev[0], st);
    }
    if (pl->nb > 0 && e == hipSuccess && a.queue)
        e = launch_zero(st, reinterpret_cast<float*>(a.queue), (size_t)kQueues * kQueueStride);
    if (pl->nb > 0 && e == hipSuccess)
        e = pl->maxd == 5 ? launch_plan_bwd_d5(dim3(pl->grid_bwd), st, a, grad_pts, slots, grad_mask)
                          : launch_plan_bwd_d7(dim3(pl->grid_bwd), st, a, grad_pts, slots, grad_mask);
    if (ev && e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (pl->nb > 0 && e == hipSuccess && (grad_mask & (NURBS_GRAD_CTRL | NURBS_GRAD_W)))
        e = pl->maxd == 5 ? launch_plan_gat_d5(st, a, slots, pl->ctx->num_cus)
                          : launch_plan_gat_d7(st, a, slots, pl->ctx->num_cus);
    if (ev && e == hipSuccess) e = hipEventRecord(ev[2], st);
    if (e == hipSuccess)
        e = pl->maxd == 5
                ? launch_plan_fin_d5(dim3((pl->nfin + kWavesPerWG - 1) / kWavesPerWG), st, a, slots, grad_ctrl,
                                     grad_w, grad_ku, grad_kv, grad_mask)
                : launch_plan_fin_d7(dim3((pl->nfin + kWavesPerWG - 1) / kWavesPerWG), st, a, slots, grad_ctrl,
                                     grad_w, grad_ku, grad_kv, grad_mask);
    if (ev && e == hipSuccess) e = hipEventRecord(ev[3], st);
    if (e != hipSuccess) return hip_fail(pl->ctx, e, "launch plan backward");
    return NURBS_OK;
}

int nurbs_plan_set_timing(nurbs_plan* pl, int max_calls) {
    if (!pl || max_calls < 0) return fail(pl ? pl->ctx : nullptr, NURBS_EINVAL, "bad arguments");
    trace_free(pl);
    if (max_calls == 0) return NURBS_OK;
    pl->ev_f.resize(2 * (size_t)max_calls);
    pl->ev_b.resize(4 * (size_t)max_calls);
    for (auto* v : {&pl->ev_f, &pl->ev_b})
        for (hipEvent_t& e : *v) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) {
                e = nullptr;
                trace_free(pl);
                return hip_fail(pl->ctx, r, "hipEventCreate");
            }
        }
    pl->trace_slots = max_calls;
    return NURBS_OK;
}

int nurbs_plan_read_timing(nurbs_plan* pl, float* fwd, int* n_fwd, float* bwd, float* gat, float* fin, int* n_bwd) {
    if (!pl) return fail(nullptr, NURBS_EINVAL, "plan is NULL");
    if (pl->trace_slots == 0) return fail(pl->ctx, NURBS_EINVAL, "timing is off");
    auto span = [&](std::vector<hipEvent_t>& ev, int per, long long calls, int j0, int j1, float* out,
                    int* n) -> hipError_t {
        const long long cnt = std::min<long long>(calls, pl->trace_slots);
        for (long long c = 0; c < cnt; ++c) {
            const long long call = calls - cnt + c;
            hipEvent_t* e = &ev[per * (size_t)(call % pl->trace_slots)];
            hipError_t r = hipEventSynchronize(e[j1]);
            float ms = 0.f;
            if (r == hipSuccess) r = hipEventElapsedTime(&ms, e[j0], e[j1]);
            if (r != hipSuccess) return r;
            if (out) out[c] = ms;
        }
        if (n) *n = (int)cnt;
        return hipSuccess;
    };
    hipError_t r = span(pl->ev_f, 2, pl->calls_f, 0, 1, fwd, n_fwd);
    if (r == hipSuccess) r = span(pl->ev_b, 4, pl->calls_b, 0, 1, bwd, n_bwd);
    if (r == hipSuccess) r = span(pl->ev_b, 4, pl->calls_b, 1, 2, gat, nullptr);
    if (r == hipSuccess) r = span(pl->ev_b, 4, pl->calls_b, 2, 3, fin, nullptr);
    return r ? hip_fail(pl->ctx, r, "read timing events") : NURBS_OK;
}

// --------------------------------------------------------------------------
// test exports and device errors
// --------------------------------------------------------------------------
int nurbs_find_spans(const float* knots, int n_knots, int p, const float* x, int nx, int32_t* spans, void* stream) {
    if (p < 1 || p > NURBS_MAX_DEGREE) return fail(nullptr, NURBS_EDEGREE, "degree");
    if (n_knots < 2 * p + 2 || nx < 0 || !knots || (nx > 0 && (!x || !spans)))
        return fail(nullptr, NURBS_EINVAL, "bad arguments");
    if (nx == 0) return NURBS_OK;
    hipError_t e = launch_spans(p, reinterpret_cast<hipStream_t>(stream), knots, n_knots, x, nx, spans, nullptr);
    return e ? hip_fail(nullptr, e, "launch k_spans") : NURBS_OK;
}

int nurbs_basis(const float* knots, int n_knots, int p, const float* x, int nx, float* N, void* stream) {
    if (p < 1 || p > NURBS_MAX_DEGREE) return fail(nullptr, NURBS_EDEGREE, "degree");
    if (n_knots < 2 * p + 2 || nx < 0 || !knots || (nx > 0 && (!x || !N)))
        return fail(nullptr, NURBS_EINVAL, "bad arguments");
    if (nx == 0) return NURBS_OK;
    hipError_t e = launch_spans(p, reinterpret_cast<hipStream_t>(stream), knots, n_knots, x, nx, nullptr, N);
    return e ? hip_fail(nullptr, e, "launch k_spans") : NURBS_OK;
}

int nurbs_read_device_error(const void* ws, void* stream, int* code) {
    if (!ws || !code) return fail(nullptr, NURBS_EINVAL, "bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int v = 0;
    hipError_t e = hipMemcpyAsync(&v, ws, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemsetAsync(const_cast<void*>(ws), 0, sizeof(int), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(nullptr, e, "read device error");
    *code = v;
    return NURBS_OK;
}

}  // extern "C"
