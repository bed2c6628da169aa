// Surfaces evaluated at scattered parameter pairs (u_k, v_k) on gfx950:
// eq. NURBS at each pair, with no tensor-product structure to share (the
// grids of Sec. 3.1 are the special case of all pairs of two lists).
//
// Forward (k_uv_fwd): one lane per pair -- both spans by binary search in
// LDS-staged knots, the p+1 and q+1 basis values, the (p+1)(q+1)-term
// homogeneous sum from the control net (staged in LDS as (x, y, z, w) per
// control point when it fits, else read through the caches), the rational
// divide; optionally dS/du, dS/dv (Appendix A, eq. NURBSuDerivative1).
//
// Backward: per pair, with g = dL/dS, W = S'_w and R_ij = N_i N_j / W,
//   dL/dP_ij += R_ij w_ij g                       (eq. NURBSuDerivative4)
//   dL/dw_ij += R_ij (P_ij - S) . g               (eq. NURBSvDerivative5)
//   e_i = sum_j N_j w_ij (P_ij - S) . g / W = dL/dN_i(u)  (eq. NURBSvDerivative6)
// and f_j likewise, through the knot adjoint of the recursion (Sec. 3.2.1).
// The pairs come in any order, so one control point collects terms from
// pairs anywhere in the input.  They are summed exactly instead of in a
// fixed order: k_uv_max finds, per surface and gradient tensor, the largest
// magnitude of a single term; k_uv_acc recomputes every term, rounds it to a
// multiple of 2^-s, with 2^s chosen so that npts times the largest term
// stays below 2^62, and adds it as a 64-bit integer (LDS atomics into a
// per-workgroup copy of the surface's accumulators when they fit in 58 KiB,
// then one global atomic per non-zero entry; global atomics otherwise).
// Integer addition is exact and associative, so the sums do not depend on
// the order the atomics land in: results are bitwise reproducible, with no
// float atomics.  k_uv_fin divides by 2^s.  The rounding error per term is
// at most npts * max|term| * 2^-63, far below that of a float32 sum.
#include "device.hpp"
#include "launch.hpp"
#include "../../include/nurbsdiff.h"

#include <algorithm>

namespace nd {
namespace {

// The basis with a runtime degree d <= DM and its knot adjoint.
template <int DM>
__device__ __forceinline__ void knot_adjoint_rt(const float* __restrict__ U, int k, float x, int d,
                                                const float e[DM + 1], float gU[2 * DM + 2]) {
#pragma unroll
    for (int t = 0; t < 2 * DM + 2; ++t) gU[t] = 0.f;
    switch (d) {
#define ND_KA(D)                                                          \
    case D:                                                               \
        if constexpr (D <= DM) {                                          \
            float ee[D + 1], gg[2 * D + 2];                               \
            _Pragma("unroll") for (int r = 0; r <= D; ++r) ee[r] = e[r];  \
            basis_knot_adjoint<D>(U, k, x, ee, gg);                       \
            _Pragma("unroll") for (int t = 0; t < 2 * D + 2; ++t) gU[t] = gg[t]; \
        }                                                                 \
        break;
        ND_KA(1) ND_KA(2) ND_KA(3) ND_KA(4) ND_KA(5) ND_KA(6) ND_KA(7)
#undef ND_KA
        default: break;
    }
}

template <int DM>
__device__ __forceinline__ int basis_d1_rt(const float* __restrict__ U, int nc, float x, int d, float N[DM + 1],
                                           float dN[DM + 1]) {
#pragma unroll
    for (int r = 0; r <= DM; ++r) N[r] = dN[r] = 0.f;
    int k = 0;
    switch (d) {
#define ND_BD(D)                                                                          \
    case D:                                                                               \
        if constexpr (D <= DM) {                                                          \
            float a[D + 1], b[D + 1];                                                     \
            k = sample_basis_d1<D>(U, nc, x, a, b);                                       \
            _Pragma("unroll") for (int r = 0; r <= D; ++r) { N[r] = a[r]; dN[r] = b[r]; } \
        }                                                                                 \
        break;
        ND_BD(1) ND_BD(2) ND_BD(3) ND_BD(4) ND_BD(5) ND_BD(6) ND_BD(7)
#undef ND_BD
        default: break;
    }
    return k;
}

// One surface of the batch, knots in LDS.
struct UvSurf {
    const float* __restrict__ ctrl;
    const float* __restrict__ w;
    const float* ku;  // LDS
    const float* kv;  // LDS
    const float4* net;  // LDS copy of (x, y, z, w) per control point, or NULL (read ctrl, w)
    const float* __restrict__ uv;
    int p, q, nu_c, nv_c, npts;
};

// control point ij as (x, y, z, w): from the LDS copy (NET) or from ctrl, w.
// Two compiled paths, so that the LDS reads stay LDS reads (one path with a
// run-time choice let the compiler merge both into generic-address loads).
template <bool NET>
__device__ __forceinline__ float4 net_at(const UvSurf& s, int ij) {
    if constexpr (NET) {
        return s.net[ij];
    } else {
        const float* c = s.ctrl + 3 * (size_t)ij;
        return make_float4(c[0], c[1], c[2], s.w[ij]);
    }
}

// Stage the surface's net in LDS (dst: ncp float4); every thread of the
// workgroup takes part, and the caller synchronises.
__device__ __forceinline__ void stage_net(const UvSurf& s, float4* dst) {
    const int ncp = s.nu_c * s.nv_c;
    for (int i = threadIdx.x; i < ncp; i += kWG) {
        const float* c = s.ctrl + 3 * (size_t)i;
        dst[i] = make_float4(c[0], c[1], c[2], s.w[i]);
    }
}

__device__ __forceinline__ UvSurf uv_surf(const UvArgs& a, int b, float* lku, float* lkv) {
    UvSurf s;
    const size_t cp = (size_t)a.nu_c * a.nv_c;
    const int nU = a.nu_c + a.p + 1, nV = a.nv_c + a.q + 1;
    s.ctrl = a.ctrl + (size_t)b * cp * 3;
    s.w = a.w + (size_t)b * cp;
    const float* gku = a.ku + (size_t)b * nU;
    const float* gkv = a.kv + (size_t)b * nV;
    for (int i = threadIdx.x; i < nU; i += kWG) lku[i] = gku[i];
    for (int i = threadIdx.x; i < nV; i += kWG) lkv[i] = gkv[i];
    s.ku = lku;
    s.kv = lkv;
    s.net = nullptr;
    s.uv = a.uv + (a.uv_shared ? 0 : (size_t)b * a.npts * 2);
    s.p = a.p;
    s.q = a.q;
    s.nu_c = a.nu_c;
    s.nv_c = a.nv_c;
    s.npts = a.npts;
    return s;
}

// Data checks (NURBS_VALIDATE): knots and weights by the surface's first
// workgroup, the parameters of each workgroup's pairs by that workgroup.
__device__ void uv_validate(const UvArgs& a, const UvSurf& s, int k0, int k1) {
    const int t = threadIdx.x;
    const int nU = s.nu_c + s.p + 1, nV = s.nv_c + s.q + 1;
    bool bad_k = false, bad_w = false, bad_d = false;
    if (blockIdx.x == 0) {
        for (int i = t; i + 1 < nU; i += kWG) bad_k |= !(s.ku[i] <= s.ku[i + 1]);
        for (int i = t; i + 1 < nV; i += kWG) bad_k |= !(s.kv[i] <= s.kv[i + 1]);
        if (t == 0)
            bad_k |= !(s.ku[s.p] < s.ku[s.p + 1]) || !(s.ku[s.nu_c - 1] < s.ku[s.nu_c]) ||
                     !(s.kv[s.q] < s.kv[s.q + 1]) || !(s.kv[s.nv_c - 1] < s.kv[s.nv_c]);
        for (int i = t; i < s.nu_c * s.nv_c; i += kWG) bad_w |= !(s.w[i] > 0.f);
    }
    const float ulo = s.ku[s.p], uhi = s.ku[s.nu_c], vlo = s.kv[s.q], vhi = s.kv[s.nv_c];
    for (int k = k0 + t; k < k1; k += kWG) {
        const float u = s.uv[2 * (size_t)k], v = s.uv[2 * (size_t)k + 1];
        bad_d |= !(u >= ulo && u <= uhi && v >= vlo && v <= vhi);
    }
    if (bad_k) atomicCAS(a.err, 0, NURBS_EKNOTS);
    if (bad_w) atomicCAS(a.err, 0, NURBS_EWEIGHTS);
    if (bad_d) atomicCAS(a.err, 0, NURBS_EDOMAIN);
}

// Span, basis and the homogeneous sum at one pair.
template <int PM, int QM>
struct UvPoint {
    int ku, kv;
    float u, v;  // clamped parameters
    float Nu[PM + 1], Nv[QM + 1];
    float4 A;    // homogeneous sum (x w, y w, z w, w)
};

template <int PM, int QM, bool NET>
__device__ __forceinline__ void uv_point(const UvSurf& s, int k, UvPoint<PM, QM>& o) {
    const float2 uv = *reinterpret_cast<const float2*>(s.uv + 2 * (size_t)k);
    o.u = clamp_param(s.ku, s.p, s.nu_c - 1, uv.x);
    o.v = clamp_param(s.kv, s.q, s.nv_c - 1, uv.y);
    o.ku = sample_basis_rt<PM>(s.ku, s.nu_c, uv.x, s.p, o.Nu);
    o.kv = sample_basis_rt<QM>(s.kv, s.nv_c, uv.y, s.q, o.Nv);
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int r = 0; r <= PM; ++r) {
        if (r > s.p) break;
        float4 R = make_float4(0.f, 0.f, 0.f, 0.f);
        const int row = (o.ku - s.p + r) * s.nv_c + (o.kv - s.q);
#pragma unroll
        for (int h = 0; h <= QM; ++h) {
            if (h > s.q) break;
            const float4 c = net_at<NET>(s, row + h);
            R = fma4(o.Nv[h], make_float4(c.x * c.w, c.y * c.w, c.z * c.w, c.w), R);
        }
        A = fma4(o.Nu[r], R, A);
    }
    o.A = A;
}

// --------------------------------------------------------------------------
// forward
// --------------------------------------------------------------------------
template <int PM, int QM, bool DER, bool NET>
__device__ __forceinline__ void uv_fwd_range(const UvSurf& s, int b, int k0, int k1, float* __restrict__ pts,
                                             float* __restrict__ du, float* __restrict__ dv) {
    for (int k = k0 + (int)threadIdx.x; k < k1; k += kWG) {
    const size_t o = ((size_t)b * s.npts + k) * 3;
    if constexpr (!DER) {
        UvPoint<PM, QM> pt;
        uv_point<PM, QM, NET>(s, k, pt);
        const float inv = recip_fast(pt.A.w);
        store3(pts + o, pt.A.x * inv, pt.A.y * inv, pt.A.z * inv);
    } else {
        // S, S_u = (A_u - S W_u) / W, S_v likewise
        const float2 uv = *reinterpret_cast<const float2*>(s.uv + 2 * (size_t)k);
        float Nu[PM + 1], dNu[PM + 1], Nv[QM + 1], dNv[QM + 1];
        const int ku = basis_d1_rt<PM>(s.ku, s.nu_c, uv.x, s.p, Nu, dNu);
        const int kv = basis_d1_rt<QM>(s.kv, s.nv_c, uv.y, s.q, Nv, dNv);
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), Au = A, Av = A;
#pragma unroll
        for (int r = 0; r <= PM; ++r) {
            if (r > s.p) break;
            float4 R = make_float4(0.f, 0.f, 0.f, 0.f), Rv = R;
            const int row = (ku - s.p + r) * s.nv_c + (kv - s.q);
#pragma unroll
            for (int h = 0; h <= QM; ++h) {
                if (h > s.q) break;
                const float4 c = net_at<NET>(s, row + h);
                const float4 pw = make_float4(c.x * c.w, c.y * c.w, c.z * c.w, c.w);
                R = fma4(Nv[h], pw, R);
                Rv = fma4(dNv[h], pw, Rv);
            }
            A = fma4(Nu[r], R, A);
            Au = fma4(dNu[r], R, Au);
            Av = fma4(Nu[r], Rv, Av);
        }
        const float inv = recip(A.w);
        const float sx = A.x * inv, sy = A.y * inv, sz = A.z * inv;
        if (pts) store3(pts + o, sx, sy, sz);
        if (du) store3(du + o, (Au.x - sx * Au.w) * inv, (Au.y - sy * Au.w) * inv, (Au.z - sz * Au.w) * inv);
        if (dv) store3(dv + o, (Av.x - sx * Av.w) * inv, (Av.y - sy * Av.w) * inv, (Av.z - sz * Av.w) * inv);
    }
    }
}

template <int PM, int QM, bool DER>
__global__ void __launch_bounds__(kWG) k_uv_fwd(UvArgs a, float* __restrict__ pts, float* __restrict__ du,
                                               float* __restrict__ dv) {
    extern __shared__ float4 lnet[];
    __shared__ float lku[kWG], lkv[kWG];
    const int b = blockIdx.y;
    UvSurf s = uv_surf(a, b, lku, lkv);
    if (a.lds_net) {
        stage_net(s, lnet);
        s.net = lnet;
    }
    __syncthreads();
    const int k0 = blockIdx.x * a.fchunk, k1 = min(s.npts, k0 + a.fchunk);
    if (a.err) uv_validate(a, s, k0, k1);
    if (a.lds_net) uv_fwd_range<PM, QM, DER, true>(s, b, k0, k1, pts, du, dv);
    else uv_fwd_range<PM, QM, DER, false>(s, b, k0, k1, pts, du, dv);
}

// --------------------------------------------------------------------------
// backward
// --------------------------------------------------------------------------
// Accumulator layout per surface (64-bit integers): control point ij at
// [4 ij .. 4 ij + 3] = (dP xyz, dw), then nU entries for ku, then nV for kv.
// Gradient classes: 0 dP, 1 dw, 2 dU, 3 dV.

// Every term of one pair, handed to emit(class, accumulator index, value).
template <int PM, int QM, bool NET, class Emit>
__device__ __forceinline__ void uv_terms(const UvSurf& s, int k, const float* __restrict__ gpts, unsigned mask,
                                         Emit& emit) {
    UvPoint<PM, QM> pt;
    uv_point<PM, QM, NET>(s, k, pt);
    const float inv = recip(pt.A.w);
    const float S0 = pt.A.x * inv, S1 = pt.A.y * inv, S2 = pt.A.z * inv;
    const float* gp = gpts + 3 * (size_t)k;
    const float g0 = gp[0], g1 = gp[1], g2 = gp[2];
    const bool want_pw = (mask & (NURBS_GRAD_CTRL | NURBS_GRAD_W)) != 0;
    const bool want_ku = (mask & NURBS_GRAD_KU) != 0, want_kv = (mask & NURBS_GRAD_KV) != 0;
    float e[PM + 1], f[QM + 1];
#pragma unroll
    for (int r = 0; r <= PM; ++r) e[r] = 0.f;
#pragma unroll
    for (int h = 0; h <= QM; ++h) f[h] = 0.f;
    const int nU = s.nu_c + s.p + 1;
#pragma unroll
    for (int r = 0; r <= PM; ++r) {
        if (r > s.p) break;
        const int row = (pt.ku - s.p + r) * s.nv_c + (pt.kv - s.q);
#pragma unroll
        for (int h = 0; h <= QM; ++h) {
            if (h > s.q) break;
            const int ij = row + h;
            const float4 c = net_at<NET>(s, ij);
            const float wt = c.w;
            float pg = (c.x - S0) * g0;
            pg = __builtin_fmaf(c.y - S1, g1, pg);
            pg = __builtin_fmaf(c.z - S2, g2, pg);
            if (want_pw) {
                const float nn = pt.Nu[r] * pt.Nv[h] * inv;
                const float nw = nn * wt;
                if (mask & NURBS_GRAD_CTRL) {
                    emit(0, 4 * ij, nw * g0);
                    emit(0, 4 * ij + 1, nw * g1);
                    emit(0, 4 * ij + 2, nw * g2);
                }
                if (mask & NURBS_GRAD_W) emit(1, 4 * ij + 3, nn * pg);
            }
            const float t = wt * pg * inv;
            e[r] = __builtin_fmaf(pt.Nv[h], t, e[r]);
            f[h] = __builtin_fmaf(pt.Nu[r], t, f[h]);
        }
    }
    const int base_u = 4 * s.nu_c * s.nv_c, base_v = base_u + nU;
    if (want_ku) {
        float gU[2 * PM + 2];
        knot_adjoint_rt<PM>(s.ku, pt.ku, pt.u, s.p, e, gU);
#pragma unroll
        for (int t = 0; t < 2 * PM + 2; ++t)
            if (t < 2 * s.p + 2) emit(2, base_u + pt.ku - s.p + t, gU[t]);
    }
    if (want_kv) {
        float gV[2 * QM + 2];
        knot_adjoint_rt<QM>(s.kv, pt.kv, pt.v, s.q, f, gV);
#pragma unroll
        for (int t = 0; t < 2 * QM + 2; ++t)
            if (t < 2 * s.q + 2) emit(3, base_v + pt.kv - s.q + t, gV[t]);
    }
}

struct EmitMax {
    float m[4];
    __device__ void operator()(int c, int, float v) { m[c] = fmaxf(m[c], fabsf(v)); }
};

// per surface: the largest |term| of each class, as float bits (max of
// non-negative floats = max of their bit patterns, an exact integer max)
template <int PM, int QM>
__global__ void __launch_bounds__(kWG) k_uv_max(UvArgs a, const float* __restrict__ gpts, unsigned mask,
                                               unsigned* __restrict__ maxbits) {
    extern __shared__ float4 lnet[];
    __shared__ float lku[kWG], lkv[kWG];
    const int b = blockIdx.y;
    UvSurf s = uv_surf(a, b, lku, lkv);
    if (a.lds_net) {
        stage_net(s, lnet);
        s.net = lnet;
    }
    __syncthreads();
    const float* g = gpts + (size_t)b * s.npts * 3;
    EmitMax em{{0.f, 0.f, 0.f, 0.f}};
    const int k0 = blockIdx.x * a.chunk, k1 = min(s.npts, k0 + a.chunk);
    if (a.err) uv_validate(a, s, k0, k1);
    if (a.lds_net)
        for (int k = k0 + (int)threadIdx.x; k < k1; k += kWG) uv_terms<PM, QM, true>(s, k, g, mask, em);
    else
        for (int k = k0 + (int)threadIdx.x; k < k1; k += kWG) uv_terms<PM, QM, false>(s, k, g, mask, em);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float v = em.m[c];
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) v = fmaxf(v, __shfl_xor(v, d));
        if (lane_id() == 0 && v > 0.f) atomicMax(maxbits + 4 * b + c, __float_as_uint(v));
    }
}

// 2^s for a class: the largest power of two with npts * maxterm * 2^s <= 2^62
__device__ __forceinline__ double fix_scale(unsigned bits, int npts) {
    const float m = __uint_as_float(bits);
    if (!(m > 0.f)) return 1.0;
    int e;
    frexp((double)m * (double)max(npts, 1), &e);  // product < 2^e
    return ldexp(1.0, 62 - e);
}

template <bool LDS>
struct EmitAcc {
    double sc[4];
    unsigned long long* acc;  // the workgroup's LDS copy (LDS) or the global accumulators
    __device__ void operator()(int c, int i, float v) {
        const long long q = __double2ll_rn((double)v * sc[c]);
        if (q == 0) return;
        if constexpr (LDS) {
            extern __shared__ unsigned long long lacc[];
            atomicAdd(lacc + i, (unsigned long long)q);
        } else {
            atomicAdd(acc + i, (unsigned long long)q);
        }
    }
};

template <int PM, int QM>
__global__ void __launch_bounds__(kWG) k_uv_acc(UvArgs a, const float* __restrict__ gpts, unsigned mask,
                                               const unsigned* __restrict__ maxbits,
                                               unsigned long long* __restrict__ acc_all) {
    extern __shared__ unsigned long long lacc[];
    __shared__ float lku[kWG], lkv[kWG];
    const int b = blockIdx.y;
    UvSurf s = uv_surf(a, b, lku, lkv);
    const int nacc = a.nacc;
    unsigned long long* gacc = acc_all + (size_t)b * nacc;
    if (a.lds_acc)
        for (int i = threadIdx.x; i < nacc; i += kWG) lacc[i] = 0ull;
    if (a.lds_net) {  // the net after the accumulators, at a 16-byte boundary
        float4* lnet = reinterpret_cast<float4*>(lacc + (a.lds_acc ? ((nacc + 1) & ~1) : 0));
        stage_net(s, lnet);
        s.net = lnet;
    }
    __syncthreads();
    double sc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) sc[c] = fix_scale(maxbits[4 * b + c], s.npts);
    const float* g = gpts + (size_t)b * s.npts * 3;
    const int k0 = blockIdx.x * a.chunk, k1 = min(s.npts, k0 + a.chunk);
    if (a.lds_acc) {
        EmitAcc<true> em{{sc[0], sc[1], sc[2], sc[3]}, nullptr};
        if (a.lds_net)
            for (int k = k0 + (int)threadIdx.x; k < k1; k += kWG) uv_terms<PM, QM, true>(s, k, g, mask, em);
        else
            for (int k = k0 + (int)threadIdx.x; k < k1; k += kWG) uv_terms<PM, QM, false>(s, k, g, mask, em);
    } else {
        EmitAcc<false> em{{sc[0], sc[1], sc[2], sc[3]}, gacc};
        if (a.lds_net)
            for (int k = k0 + (int)threadIdx.x; k < k1; k += kWG) uv_terms<PM, QM, true>(s, k, g, mask, em);
        else
            for (int k = k0 + (int)threadIdx.x; k < k1; k += kWG) uv_terms<PM, QM, false>(s, k, g, mask, em);
    }
    if (a.lds_acc) {
        __syncthreads();
        for (int i = threadIdx.x; i < nacc; i += kWG) {
            const unsigned long long v = lacc[i];
            if (v) atomicAdd(gacc + i, v);
        }
    }
}

__global__ void __launch_bounds__(kWG) k_uv_fin(UvArgs a, const unsigned* __restrict__ maxbits,
                                               const unsigned long long* __restrict__ acc_all, unsigned mask,
                                               float* __restrict__ gc, float* __restrict__ gw,
                                               float* __restrict__ gku, float* __restrict__ gkv) {
    const long long t = (long long)blockIdx.x * kWG + threadIdx.x;
    const int nacc = a.nacc;
    if (t >= (long long)a.B * nacc) return;
    const int b = (int)(t / nacc), i = (int)(t - (long long)b * nacc);
    const int ncp = a.nu_c * a.nv_c, nU = a.nu_c + a.p + 1;
    const long long v = (long long)acc_all[t];
    int c;
    if (i < 4 * ncp) c = (i & 3) == 3 ? 1 : 0;
    else if (i < 4 * ncp + nU) c = 2;
    else c = 3;
    const float x = (float)((double)v / fix_scale(maxbits[4 * b + c], a.npts));
    if (i < 4 * ncp) {
        const int ij = i >> 2, comp = i & 3;
        if (comp < 3) {
            if (mask & NURBS_GRAD_CTRL) gc[((size_t)b * ncp + ij) * 3 + comp] = x;
        } else if (mask & NURBS_GRAD_W) {
            gw[(size_t)b * ncp + ij] = x;
        }
    } else if (i < 4 * ncp + nU) {
        if (mask & NURBS_GRAD_KU) gku[(size_t)b * nU + (i - 4 * ncp)] = x;
    } else if (mask & NURBS_GRAD_KV) {
        gkv[(size_t)b * (a.nv_c + a.q + 1) + (i - 4 * ncp - nU)] = x;
    }
}

template <int PM, int QM>
hipError_t uv_fwd_launch(const UvArgs& a, hipStream_t st, float* pts, float* du, float* dv) {
    const dim3 grid((unsigned)((a.npts + a.fchunk - 1) / a.fchunk), (unsigned)a.B);
    const size_t lds = a.lds_net ? sizeof(float4) * (size_t)a.nu_c * a.nv_c : 0;
    if (du || dv) hipLaunchKernelGGL((k_uv_fwd<PM, QM, true>), grid, dim3(kWG), lds, st, a, pts, du, dv);
    else hipLaunchKernelGGL((k_uv_fwd<PM, QM, false>), grid, dim3(kWG), lds, st, a, pts, du, dv);
    return hipGetLastError();
}

template <int PM, int QM>
hipError_t uv_bwd_launch(const UvArgs& a, hipStream_t st, const float* gpts, unsigned mask, unsigned* maxbits,
                         unsigned long long* acc, float* gc, float* gw, float* gku, float* gkv) {
    hipError_t e = launch_zero(st, reinterpret_cast<float*>(maxbits), (size_t)a.B * 4);
    if (e == hipSuccess) e = launch_zero(st, reinterpret_cast<float*>(acc), (size_t)a.B * a.nacc * 2);
    if (e != hipSuccess) return e;
    if (a.npts > 0) {  // no pairs: the zeroed accumulators give zero gradients
        const dim3 grid((unsigned)((a.npts + a.chunk - 1) / a.chunk), (unsigned)a.B);
        const size_t net = a.lds_net ? sizeof(float4) * (size_t)a.nu_c * a.nv_c : 0;
        hipLaunchKernelGGL((k_uv_max<PM, QM>), grid, dim3(kWG), net, st, a, gpts, mask, maxbits);
        const size_t lds = (a.lds_acc ? sizeof(unsigned long long) * (size_t)((a.nacc + 1) & ~1) : 0) + net;
        hipLaunchKernelGGL((k_uv_acc<PM, QM>), grid, dim3(kWG), lds, st, a, gpts, mask, maxbits, acc);
    }
    const long long items = (long long)a.B * a.nacc;
    hipLaunchKernelGGL(k_uv_fin, dim3((unsigned)((items + kWG - 1) / kWG)), dim3(kWG), 0, st, a, maxbits, acc, mask,
                       gc, gw, gku, gkv);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_uv_fwd(const UvArgs& a, hipStream_t st, float* pts, float* du, float* dv) {
    return (a.p <= 3 && a.q <= 3) ? uv_fwd_launch<3, 3>(a, st, pts, du, dv) : uv_fwd_launch<7, 7>(a, st, pts, du, dv);
}

hipError_t launch_uv_bwd(const UvArgs& a, hipStream_t st, const float* gpts, unsigned mask, unsigned* maxbits,
                         unsigned long long* acc, float* gc, float* gw, float* gku, float* gkv) {
    return (a.p <= 3 && a.q <= 3) ? uv_bwd_launch<3, 3>(a, st, gpts, mask, maxbits, acc, gc, gw, gku, gkv)
                                  : uv_bwd_launch<7, 7>(a, st, gpts, mask, maxbits, acc, gc, gw, gku, gkv);
}

}  // namespace nd
