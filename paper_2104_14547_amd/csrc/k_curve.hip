// Rational B-spline curves in the plane and in space on gfx950.
//
//   C(u) = sum_i N_i^p(u) w_i P_i / sum_i N_i^p(u) w_i
//
// is eq. NURBS with one parametric direction: NURBS-Diff (Sec. 3) gets its
// curve layer from the surface formulas by dropping a direction.  Per sample
// the forward takes the span, the p+1 non-zero basis functions (Sec. 3.1.2
// steps 1-2), the homogeneous sum and the rational divide (step 3), and on
// request dC/du = (A_u - C W_u) / W (Appendix A, eq. NURBSuDerivative1).  The
// backward is Sec. 3.2 without v: with g = dL/dC at a sample,
//   dL/dP_i += N_i w_i g / W                    (eq. NURBSuDerivative4)
//   dL/dw_i += N_i (P_i - C) . g / W            (eq. NURBSvDerivative5)
//   dL/dN_i  = w_i (P_i - C) . g / W            (eq. NURBSvDerivative6)
// and dL/dU_k from dL/dN_i through the knot adjoint of the recursion
// (Sec. 3.2.1).  dL/dw is taken directly from P_i - C (not as P . dL/dPw +
// dL/dPw_w), so no difference of two large sums is formed.
//
// Work decomposition.  A workgroup (4 waves) owns one chunk of up to
// kCurveChunk consecutive samples of one curve and stages that curve's knots
// and control polygon in LDS.  A wave handles 64 consecutive samples at a
// time, one per lane.  Backward contributions are reduced without atomics:
// when the 64 spans of a wave are non-decreasing (sorted parameters, the
// usual case), equal spans form runs of lanes and a DPP segmented scan (the
// surface backward's, one v_fmac_f32_dpp per value and step) sums each run,
// whose last lane adds the sums into the wave's LDS accumulators; an
// unsorted wave adds its lanes one after the other.  At the end of the
// chunk the four waves' accumulators are added in wave order.  A curve with
// one chunk writes its gradients directly; longer curves write one partial
// per chunk to the workspace and a finalize kernel adds the partials in
// chunk order.  Every sum has a fixed order, so results are bitwise
// reproducible.
#include "kernels.hpp"
#include "launch.hpp"
#include "../../include/nurbsdiff.h"

namespace nd {
namespace {

__device__ __forceinline__ void curve_post_error(int* err, int code) {
    if (err) atomicCAS(err, 0, code);
}

// Data checks (NURBS_VALIDATE): knots and weights by the curve's first
// chunk, parameters by every chunk.
__device__ void curve_validate(const CurveArgs& a, int p, int c, int chunk, int s0, int s1, const float* U,
                               const float* w, const float* us) {
    const int t = threadIdx.x;
    const int nU = a.nc + p + 1;
    bool bad_k = false, bad_w = false, bad_d = false;
    if (chunk == 0) {
        for (int i = t; i + 1 < nU; i += kWG) bad_k |= !(U[i] <= U[i + 1]);
        if (t == 0) bad_k |= !(U[p] < U[p + 1]) || !(U[a.nc - 1] < U[a.nc]);
        for (int i = t; i < a.nc; i += kWG) bad_w |= !(w[i] > 0.f);
    }
    const float lo = U[p], hi = U[a.nc];
    for (int s = s0 + t; s < s1; s += kWG) bad_d |= !(us[s] >= lo && us[s] <= hi);
    if (bad_k) curve_post_error(a.err, NURBS_EKNOTS);
    if (bad_w) curve_post_error(a.err, NURBS_EWEIGHTS);
    if (bad_d) curve_post_error(a.err, NURBS_EDOMAIN);
}

// (curve, chunk) of this workgroup, and the chunk's sample range
struct CurveBlock {
    int c, chunk, s0, s1;
};
__device__ __forceinline__ CurveBlock curve_block(const CurveArgs& a) {
    CurveBlock b;
    const int blk = (int)blockIdx.x;
    b.c = blk / a.nchunks;
    b.chunk = blk - b.c * a.nchunks;
    b.s0 = b.chunk * kCurveChunk;
    b.s1 = min(a.ns, b.s0 + kCurveChunk);
    return b;
}

// Stage the curve's knots and control points (xyz or xy, and the weight) in LDS.
template <int DIM>
__device__ __forceinline__ void stage_curve(const CurveArgs& a, int p, int c, float* U, float4* Pw) {
    const int nU = a.nc + p + 1;
    const float* kn = a.knots + (size_t)c * nU;
    const float* cp = a.ctrl + (size_t)c * a.nc * DIM;
    const float* w = a.w + (size_t)c * a.nc;
    for (int i = threadIdx.x; i < nU; i += kWG) U[i] = kn[i];
    for (int i = threadIdx.x; i < a.nc; i += kWG)
        Pw[i] = make_float4(cp[i * DIM], cp[i * DIM + 1], DIM == 3 ? cp[i * DIM + 2] : 0.f, w[i]);
}

// --------------------------------------------------------------------------
// forward
// --------------------------------------------------------------------------
template <int P, int DIM, bool DU>
__global__ void __launch_bounds__(kWG) k_curve_fwd(CurveArgs a, float* __restrict__ pts, float* __restrict__ du) {
    __shared__ float U[kWG];
    __shared__ float4 Pw[kWG];
    const CurveBlock b = curve_block(a);
    stage_curve<DIM>(a, P, b.c, U, Pw);
    __syncthreads();
    const float* us = a.us + (a.u_shared ? 0 : (size_t)b.c * a.ns);
    if (a.err) curve_validate(a, P, b.c, b.chunk, b.s0, b.s1, U, a.w + (size_t)b.c * a.nc, us);
    const size_t base = (size_t)b.c * a.ns;
    for (int s = b.s0 + (int)threadIdx.x; s < b.s1; s += kWG) {
        const float x = clamp_param(U, P, a.nc - 1, us[s]);
        const int k = find_span(U, P, a.nc - 1, x);
        float N[P + 1], dN[P + 1];
        if constexpr (DU) basis_d1_f32<P>(U, k, x, N, dN);
        else basis_f32<P>(U, k, x, N);
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), Au = A;
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            const float4 q = Pw[k - P + r];
            const float4 hq = make_float4(q.x * q.w, q.y * q.w, q.z * q.w, q.w);
            A = fma4(N[r], hq, A);
            if constexpr (DU) Au = fma4(dN[r], hq, Au);
        }
        const float inv = recip_fast(A.w);
        const float cx = A.x * inv, cy = A.y * inv, cz = A.z * inv;
        float* o = pts + (base + s) * DIM;
        if constexpr (DIM == 3) store3(o, cx, cy, cz);
        else *reinterpret_cast<float2*>(o) = make_float2(cx, cy);
        if constexpr (DU) {
            float* d = du + (base + s) * DIM;
            const float ex = (Au.x - cx * Au.w) * inv, ey = (Au.y - cy * Au.w) * inv;
            if constexpr (DIM == 3) store3(d, ex, ey, (Au.z - cz * Au.w) * inv);
            else *reinterpret_cast<float2*>(d) = make_float2(ex, ey);
        }
    }
}

// --------------------------------------------------------------------------
// backward
// --------------------------------------------------------------------------

// per-wave accumulators: control point i -> (dL/dP_i xyz, dL/dw_i); knot t -> dL/dU_t
struct CurveAcc {
    float4 cp[kWG];
    float kn[kWG];
};

template <int P, int DIM>
__global__ void __launch_bounds__(kWG) k_curve_bwd(CurveArgs a, const float* __restrict__ gpts,
                                                   float* __restrict__ gctrl, float* __restrict__ gw,
                                                   float* __restrict__ gk, float* __restrict__ part,
                                                   unsigned mask) {
    __shared__ float U[kWG];
    __shared__ float4 Pw[kWG];
    __shared__ CurveAcc acc[kWavesPerWG];
    const CurveBlock b = curve_block(a);
    const int nU = a.nc + P + 1;
    stage_curve<DIM>(a, P, b.c, U, Pw);
    for (int wv = 0; wv < kWavesPerWG; ++wv)
        for (int i = threadIdx.x; i < kWG; i += kWG) {
            acc[wv].cp[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            acc[wv].kn[i] = 0.f;
        }
    __syncthreads();
    const float* us = a.us + (a.u_shared ? 0 : (size_t)b.c * a.ns);
    if (a.err) curve_validate(a, P, b.c, b.chunk, b.s0, b.s1, U, a.w + (size_t)b.c * a.nc, us);
    const bool want_k = (mask & NURBS_GRAD_KU) != 0;
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    CurveAcc& A = acc[wv];
    const float* g0 = gpts + (size_t)b.c * a.ns * DIM;
    constexpr int kSentinel = 1 << 20;  // span of lanes past the chunk end
    for (int base = b.s0 + wv * kWave; base < b.s1; base += kWG) {
        const int s = base + lane;
        const bool act = s < b.s1;
        // per control point r of the sample's span: (dL/dP xyz, dL/dw)
        float4 c4[P + 1];
        float gU[2 * P + 2];
        int k = kSentinel;
#pragma unroll
        for (int r = 0; r <= P; ++r) c4[r] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int t = 0; t < 2 * P + 2; ++t) gU[t] = 0.f;
        if (act) {
            const float x = clamp_param(U, P, a.nc - 1, us[s]);
            k = find_span(U, P, a.nc - 1, x);
            float N[P + 1];
            basis_f32<P>(U, k, x, N);
            float Wsum = 0.f, C[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r <= P; ++r) {
                const float4 q = Pw[k - P + r];
                const float c = N[r] * q.w;
                Wsum += c;
                C[0] = __builtin_fmaf(c, q.x, C[0]);
                C[1] = __builtin_fmaf(c, q.y, C[1]);
                if constexpr (DIM == 3) C[2] = __builtin_fmaf(c, q.z, C[2]);
            }
            const float inv = recip(Wsum);
#pragma unroll
            for (int x2 = 0; x2 < DIM; ++x2) C[x2] *= inv;
            const float g[3] = {g0[(size_t)s * DIM], g0[(size_t)s * DIM + 1],
                                DIM == 3 ? g0[(size_t)s * DIM + 2] : 0.f};
            float e[P + 1];
#pragma unroll
            for (int r = 0; r <= P; ++r) {
                const float4 q = Pw[k - P + r];
                float pg = (q.x - C[0]) * g[0];
                pg = __builtin_fmaf(q.y - C[1], g[1], pg);
                if constexpr (DIM == 3) pg = __builtin_fmaf(q.z - C[2], g[2], pg);
                const float nw = N[r] * q.w * inv;
                c4[r] = make_float4(nw * g[0], nw * g[1], nw * g[2], N[r] * pg * inv);
                e[r] = q.w * pg * inv;
            }
            if (want_k) basis_knot_adjoint<P>(U, k, x, e, gU);
        }
        // spans non-decreasing across the wave?
        int kprev = __shfl_up(k, 1);
        if (lane == 0) kprev = k;
        const bool sorted = __ballot(k < kprev) == 0ull;
        if (sorted) {
            // runs of equal spans: DPP segmented scans, then the last lane of
            // each run adds the run's sums; for a fixed r the run ends touch
            // distinct control points
            const Runs rn = wave_runs(k);
#pragma unroll
            for (int r = 0; r <= P; ++r) seg_scan4(c4[r], rn);
            if (want_k) {
#pragma unroll
                for (int t = 0; t < 2 * P + 2; t += 2) seg_scan2(gU[t], gU[t + 1], rn);
            }
            const bool wr = rn.head && k != kSentinel;
#pragma unroll
            for (int r = 0; r <= P; ++r) {
                if (wr) {
                    float4 v = A.cp[k - P + r];
                    v.x += c4[r].x;
                    v.y += c4[r].y;
                    if constexpr (DIM == 3) v.z += c4[r].z;
                    v.w += c4[r].w;
                    A.cp[k - P + r] = v;
                }
                wave_lds_sync();
            }
            if (want_k) {
#pragma unroll
                for (int t = 0; t < 2 * P + 2; ++t) {
                    if (wr) A.kn[k - P + t] += gU[t];
                    wave_lds_sync();
                }
            }
        } else {
            // unsorted parameters: the lanes' contributions one after the
            // other, lane r (r <= P) adding the r-th control point of each
            // sample and lane t (t <= 2P+1) its t-th knot
            for (int l = 0; l < kWave; ++l) {
                const int kl = __builtin_amdgcn_readlane(k, l);
                if (kl == kSentinel) break;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int r = 0; r <= P; ++r) {
                    const float px = bcast_lane(c4[r].x, l), py = bcast_lane(c4[r].y, l);
                    const float pz = DIM == 3 ? bcast_lane(c4[r].z, l) : 0.f;
                    const float pw = bcast_lane(c4[r].w, l);
                    if (lane == r) v = make_float4(px, py, pz, pw);
                }
                if (lane <= P) {
                    float4 o = A.cp[kl - P + lane];
                    o.x += v.x;
                    o.y += v.y;
                    o.z += v.z;
                    o.w += v.w;
                    A.cp[kl - P + lane] = o;
                }
                if (want_k) {
                    float gv = 0.f;
#pragma unroll
                    for (int t = 0; t < 2 * P + 2; ++t) {
                        const float y = bcast_lane(gU[t], l);
                        if (lane == t) gv = y;
                    }
                    if (lane < 2 * P + 2) A.kn[kl - P + lane] += gv;
                }
                wave_lds_sync();
            }
        }
    }
    __syncthreads();
    // the chunk's totals, waves added in order
    const bool direct = a.nchunks == 1;
    float* pc = direct ? nullptr : part + ((size_t)b.c * a.nchunks + b.chunk) * a.part_floats;
    for (int i = threadIdx.x; i < a.nc; i += kWG) {
        float4 v = acc[0].cp[i];
#pragma unroll
        for (int w2 = 1; w2 < kWavesPerWG; ++w2) {
            const float4 o = acc[w2].cp[i];
            v.x += o.x;
            v.y += o.y;
            v.z += o.z;
            v.w += o.w;
        }
        if (direct) {
            const size_t ci = (size_t)b.c * a.nc + i;
            if (mask & NURBS_GRAD_CTRL) {
                gctrl[ci * DIM] = v.x;
                gctrl[ci * DIM + 1] = v.y;
                if constexpr (DIM == 3) gctrl[ci * DIM + 2] = v.z;
            }
            if (mask & NURBS_GRAD_W) gw[ci] = v.w;
        } else {
            reinterpret_cast<float4*>(pc)[i] = v;
        }
    }
    if (want_k) {
        for (int t = threadIdx.x; t < nU; t += kWG) {
            float v = acc[0].kn[t];
#pragma unroll
            for (int w2 = 1; w2 < kWavesPerWG; ++w2) v += acc[w2].kn[t];
            if (direct) gk[(size_t)b.c * nU + t] = v;
            else pc[4 * a.nc + t] = v;
        }
    }
}

// Multi-chunk curves: gradient entry e of curve c is the sum of its chunk
// partials in chunk order.  One thread per (curve, entry).
template <int DIM>
__global__ void __launch_bounds__(kWG) k_curve_fin(CurveArgs a, int p, const float* __restrict__ part,
                                                   float* __restrict__ gctrl, float* __restrict__ gw,
                                                   float* __restrict__ gk, unsigned mask) {
    const int nU = a.nc + p + 1;
    const int per = a.nc + nU;
    const long long id = (long long)blockIdx.x * kWG + threadIdx.x;
    if (id >= (long long)a.B * per) return;
    const int c = (int)(id / per), e = (int)(id - (long long)c * per);
    const float* pc = part + (size_t)c * a.nchunks * a.part_floats;
    if (e < a.nc) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int ch = 0; ch < a.nchunks; ++ch) {
            const float4 o = reinterpret_cast<const float4*>(pc + (size_t)ch * a.part_floats)[e];
            v.x += o.x;
            v.y += o.y;
            v.z += o.z;
            v.w += o.w;
        }
        const size_t ci = (size_t)c * a.nc + e;
        if (mask & NURBS_GRAD_CTRL) {
            gctrl[ci * DIM] = v.x;
            gctrl[ci * DIM + 1] = v.y;
            if constexpr (DIM == 3) gctrl[ci * DIM + 2] = v.z;
        }
        if (mask & NURBS_GRAD_W) gw[ci] = v.w;
    } else if (mask & NURBS_GRAD_KU) {
        const int t = e - a.nc;
        float v = 0.f;
        for (int ch = 0; ch < a.nchunks; ++ch) v += pc[(size_t)ch * a.part_floats + 4 * a.nc + t];
        gk[(size_t)c * nU + t] = v;
    }
}

template <int P, int DIM>
hipError_t curve_fwd_launch(const CurveArgs& a, hipStream_t st, float* pts, float* du) {
    const dim3 grid((unsigned)((long long)a.B * a.nchunks));
    if (du) hipLaunchKernelGGL((k_curve_fwd<P, DIM, true>), grid, dim3(kWG), 0, st, a, pts, du);
    else hipLaunchKernelGGL((k_curve_fwd<P, DIM, false>), grid, dim3(kWG), 0, st, a, pts, du);
    return hipGetLastError();
}

template <int P, int DIM>
hipError_t curve_bwd_launch(const CurveArgs& a, hipStream_t st, const float* gpts, float* gctrl, float* gw,
                            float* gk, float* part, unsigned mask) {
    const dim3 grid((unsigned)((long long)a.B * a.nchunks));
    hipLaunchKernelGGL((k_curve_bwd<P, DIM>), grid, dim3(kWG), 0, st, a, gpts, gctrl, gw, gk, part, mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.nchunks == 1) return e;
    const long long items = (long long)a.B * (2 * a.nc + P + 1);
    hipLaunchKernelGGL((k_curve_fin<DIM>), dim3((unsigned)((items + kWG - 1) / kWG)), dim3(kWG), 0, st, a, P, part,
                       gctrl, gw, gk, mask);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_curve_fwd(int p, int dim, hipStream_t st, const CurveArgs& a, float* pts, float* du) {
    switch (p * 4 + dim) {
#define C(P)                                                     \
    case P * 4 + 2: return curve_fwd_launch<P, 2>(a, st, pts, du); \
    case P * 4 + 3: return curve_fwd_launch<P, 3>(a, st, pts, du);
        C(1) C(2) C(3) C(4) C(5) C(6) C(7)
#undef C
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_curve_bwd(int p, int dim, hipStream_t st, const CurveArgs& a, const float* gpts, float* gctrl,
                            float* gw, float* gk, float* part, unsigned mask) {
    switch (p * 4 + dim) {
#define C(P)                                                                               \
    case P * 4 + 2: return curve_bwd_launch<P, 2>(a, st, gpts, gctrl, gw, gk, part, mask); \
    case P * 4 + 3: return curve_bwd_launch<P, 3>(a, st, gpts, gctrl, gw, gk, part, mask);
        C(1) C(2) C(3) C(4) C(5) C(6) C(7)
#undef C
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nd
