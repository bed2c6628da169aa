// Kernel argument blocks and launcher entry points shared by the kernel
// translation units and the host ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace nd {

// B surfaces of one shape; tile index arithmetic, no tables.
struct UniformArgs {
    const float *ctrl, *w, *ku, *kv, *us, *vs;
    int B, nu_c, nv_c, nu_s, nv_s, uv_shared;
    int ncb, nrb, rows;  // column blocks, row blocks, rows per tile
    int ntiles;
    unsigned flags;
    int* err;
    // fixed-knot tables (NULL: spans and basis are evaluated); per surface
    // at tab_u + s * tab_u_stride (stride 0: one table for the batch)
    const char *tab_u, *tab_v;
    size_t tab_u_stride, tab_v_stride;
};

// Dynamic plan schedule: tiles are dealt to kQueues queues round-robin in
// longest-first order; each queue's counter sits on its own 128-byte line
// (kQueueStride ints apart) in the plan workspace's header.
constexpr int kQueues = 16;
constexpr int kQueueStride = 32;

// Byte offset of the basis rows in a fixed-knot table of n samples (the
// n int32 spans come first).
__host__ __device__ inline size_t basis_table_split(int n) { return ((size_t)n * 4 + 255) & ~size_t(255); }

// One surface of a ragged batch, as the device sees it.
struct DevDesc {
    int p, q, nu_c, nv_c, nu_s, nv_s;
    long long ctrl_off, w_off, ku_off, kv_off, us_off, vs_off, pts_off;
    int tile_first, tile_count;  // backward tiles of this surface, natural order
    int rows;                    // rows per backward tile of this surface
    int pad;
    long long slot0;             // byte offset of its first backward slot (the others follow, equal-sized)
};

// One tile of a ragged batch.
struct DevTile {
    int surf, col0, row0, row1;
    long long slot_off;  // backward: byte offset of the tile's workspace slot
};

// Everything a wave needs to start a tile, in one record: the surface's
// shape and array offsets and the tile's range (26 words, fetched with one
// vector load, one word per lane).
struct ExecTile {
    int p, q, nu_c, nv_c, nu_s, nv_s;
    int col0, row0, row1;
    int rows;  // rows per backward tile of the surface (workspace slot layout)
    long long ctrl_off, w_off, ku_off, kv_off, us_off, vs_off, pts_off;
    long long slot_off;  // backward: byte offset of the tile's workspace slot
};
static_assert(sizeof(ExecTile) == 104, "ExecTile layout");

struct PlanArgs {
    const DevDesc* desc;
    const DevTile* tiles;     // natural order (finalize)
    const ExecTile* exec;     // execution records; wave w runs exec[wave_begin[w] .. wave_begin[w + 1])
    const ExecTile* gexec;    // backward: the same records by decreasing estimated gather work
    const int* wave_begin;    // [nwaves + 1], assigned at plan creation (static schedule)
    int* queue;               // dynamic schedule: kQueues tile counters (zeroed before the launch); NULL: static
    int ntiles;
    int nwaves;               // persistent waves in the grid (grid * kWavesPerWG)
    unsigned flags;
    int* err;
    const float *ctrl, *w, *ku, *kv, *us, *vs;
    int nsurf;             // surfaces in the plan
    const int2* fin_items; // finalize parts (surface, part), most expensive first
    int nfin;
};

// uniform batch, one entry per degree in u (defined in k_uniform_p<P>.hip)
#define ND_DECLARE_UNIFORM(P)                                                                          \
    hipError_t launch_uniform_fwd_p##P(int q, dim3 grid, hipStream_t st, const UniformArgs& a,         \
                                       float* pts);                                                    \
    hipError_t launch_uniform_der_p##P(int q, dim3 grid, hipStream_t st, const UniformArgs& a,         \
                                       float* pts, float* du, float* dv, float* nrm);                  \
    hipError_t launch_uniform_bwd_p##P(int q, dim3 grid, hipStream_t st, const UniformArgs& a,         \
                                       const float* gpts, char* slots, size_t slot_sz, unsigned mask); \
    hipError_t launch_uniform_fin_p##P(int q, dim3 grid, hipStream_t st, const UniformArgs& a,         \
                                       const char* slots, size_t slot_sz, float* gc, float* gw,        \
                                       float* gku, float* gkv, unsigned mask);
ND_DECLARE_UNIFORM(1)
ND_DECLARE_UNIFORM(2)
ND_DECLARE_UNIFORM(3)
ND_DECLARE_UNIFORM(4)
ND_DECLARE_UNIFORM(5)
ND_DECLARE_UNIFORM(6)
ND_DECLARE_UNIFORM(7)
#undef ND_DECLARE_UNIFORM

// ragged batch: persistent kernels for degree class <= 5 and <= 7
#define ND_DECLARE_PLAN(M)                                                                            \
    hipError_t launch_plan_fwd_d##M(dim3 grid, hipStream_t st, const PlanArgs& a, float* pts);        \
    hipError_t launch_plan_bwd_d##M(dim3 grid, hipStream_t st, const PlanArgs& a, const float* gpts,  \
                                    char* slots, unsigned mask);                                      \
    hipError_t launch_plan_fin_d##M(dim3 grid, hipStream_t st, const PlanArgs& a, const char* slots,  \
                                    float* gc, float* gw, float* gku, float* gkv, unsigned mask);     \
    hipError_t occupancy_plan_fwd_d##M(int* blocks_per_cu);                                           \
    hipError_t occupancy_plan_bwd_d##M(int* blocks_per_cu);                                           \
    /* gather (after the backward, before the finalize): plan tiles, uniform tiles; cus: compute units */ \
    hipError_t launch_plan_gat_d##M(hipStream_t st, const PlanArgs& a, char* slots, int cus);         \
    hipError_t launch_uniform_gat_d##M(hipStream_t st, const UniformArgs& a, int p, int q, char* slots, \
                                       size_t slot_sz, int cus);
ND_DECLARE_PLAN(5)
ND_DECLARE_PLAN(7)
#undef ND_DECLARE_PLAN

// curves: B curves of one shape (k_curve.hip)
constexpr int kCurveChunk = 2048;  // samples per workgroup
struct CurveArgs {
    const float *ctrl, *w, *knots, *us;  // [B][nc][dim], [B][nc], [B][nc+p+1], [B or 1][ns]
    int B, nc, ns, u_shared;
    int nchunks;      // workgroups per curve, ceil(ns / kCurveChunk)
    int part_floats;  // floats per chunk partial in the workspace (multi-chunk curves)
    int* err;         // device error word (NURBS_VALIDATE) or NULL
};
hipError_t launch_curve_fwd(int p, int dim, hipStream_t st, const CurveArgs& a, float* pts, float* du);
hipError_t launch_curve_bwd(int p, int dim, hipStream_t st, const CurveArgs& a, const float* gpts, float* gctrl,
                            float* gw, float* gk, float* part, unsigned mask);

// surfaces at scattered (u, v) pairs: B surfaces of one shape (k_uv.hip)
struct UvArgs {
    const float *ctrl, *w, *ku, *kv, *uv;  // uv [B or 1][npts][2]
    int B, p, q, nu_c, nv_c, npts, uv_shared;
    int chunk;    // pairs per backward workgroup
    int nacc;     // 64-bit accumulators per surface: 4 nu_c nv_c + nU + nV
    int lds_acc;  // accumulate in LDS first (nacc * 8 bytes fit)
    int lds_net;  // stage the net in LDS (16 bytes per control point, beside the accumulators)
    int fchunk;   // pairs per forward workgroup
    int* err;     // device error word (NURBS_VALIDATE) or NULL
};
constexpr int kUvLdsAccMax = 7424;                 // accumulators a workgroup keeps in LDS (58 KiB)
constexpr size_t kUvLdsDynMax = 60 * 1024 - 2048;  // dynamic LDS per workgroup (static: the knots)
hipError_t launch_uv_fwd(const UvArgs& a, hipStream_t st, float* pts, float* du, float* dv);
hipError_t launch_uv_bwd(const UvArgs& a, hipStream_t st, const float* gpts, unsigned mask, unsigned* maxbits,
                         unsigned long long* acc, float* gc, float* gw, float* gku, float* gkv);

// point-set losses (k_chamfer.hip)
struct NnSplit {
    int nranges;  // target ranges (workgroups along the target set)
    int range;    // targets per range (a multiple of 256)
};
NnSplit nn_split(int B, int n, int m, int num_cus);
hipError_t launch_nn(int dim, hipStream_t st, int B, const float* X, int n, const float* Y, int m,
                     const NnSplit& sp, int* idx, float* d2, int* pidx, float* pd2);
hipError_t launch_cd(int dim, hipStream_t st, int B, const float* P, int n, const float* Q, int m, const int* a,
                     const float* da, const int* bq, const float* db, float* out, void* state, void* part,
                     void* acc, float* gcd, float* ghd);
size_t cd_state_bytes();
size_t cd_part_bytes(int n, int m);  // per pair

// test exports
// zero n floats on stream st (a kernel, so graph capture records no memset)
hipError_t launch_zero(hipStream_t st, float* p, size_t n);
hipError_t launch_spans(int p, hipStream_t st, const float* U, int nk, const float* x, int nx, int* spans,
                        float* N);

}  // namespace nd
