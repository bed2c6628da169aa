// Device building blocks for NURBS surface evaluation on gfx950 (wave64).
//
// Span search and basis (Sec. 3.1.2 steps 1-2 of NURBS-Diff, eqs. NURBSBasis
// and BSplineBasis2), the homogeneous control point (Sec. 3.1.2 step 3), the
// reverse-mode knot derivative of the recursion (Sec. 3.2.1) and wave-level
// helpers.  Everything runs in FP32 on FP32 inputs: span search compares the
// input values exactly; every factor of the basis recursion and of its knot
// derivative is a ratio of differences of input values, so each carries a
// few ulp of relative error.  Only the per-knot sums of the knot gradient
// (long sums over samples) accumulate in FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nd {

constexpr int kWave = 64;
constexpr int kWavesPerWG = 4;
constexpr int kWG = kWave * kWavesPerWG;
constexpr int kMaxDeg = 7;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// The lane index as a value the compiler cannot see through.  Rare-path code
// (block staging, flushes) derives its addresses from it, so those addresses
// are recomputed where they are used instead of being hoisted out of the row
// loops and held in registers for the whole tile.
__device__ __forceinline__ int lane_opaque() {
    int l = __lane_id();
    asm volatile("" : "+v"(l));
    return l;
}

__device__ __forceinline__ int bcast_lane(int x, int l) {
    return __builtin_amdgcn_readlane(x, l);
}
__device__ __forceinline__ float bcast_lane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ long long uniform64(long long x) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(x & 0xffffffffll));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)x >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Wait until every global memory operation this wave issued has completed
// (s_waitcnt vmcnt(0); gfx9 encoding, expcnt and lgkmcnt left at their
// maxima).  Placed at the end of a conditional staging step, it tells the
// compiler that nothing is outstanding on any path out of the step, so no
// conservative vmcnt(0) -- which also waits for earlier stores -- is inserted
// at later uses of the staging registers inside the hot loop.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Order this wave's LDS traffic: everything before is visible to every lane
// after (LDS executes in order per wave; this stops compiler reordering).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/x from the hardware reciprocal plus one Newton-Raphson step
// (r <- r + r(1 - x r)), about 0.5 ulp for the normal range used here.
__device__ __forceinline__ float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// 1/x from the hardware reciprocal alone (1 ulp): the per-point rational
// divide, whose result is compared at 1e-5 of the surface's extent.
__device__ __forceinline__ float recip_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// q = floor(n / d) for 0 <= n < 2^16 and 1 <= d < 2^16, through the FP32
// reciprocal: the quotient's fractional part is at least 1/d away from the
// next integer, far above the rounding of the product.
__device__ __forceinline__ int small_div(int n, int d) {
    return (int)(((float)n + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

// Sums over each 16-lane DPP row, every lane of the row getting its row's
// sum, for N values at once.  Four butterfly steps in a fixed order
// (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror),
// so the result is bitwise reproducible.  Each step is one v_add_f32
// reading its other operand through DPP; the values go through the steps
// interleaved, four (or two, or one) to an asm block, so a value's next DPP
// read comes two instructions or more after its write (s_nop fills in for
// fewer than three values); each block opens with s_nop 1 for the writes
// before it.
__device__ __forceinline__ void row16_sum4(float& a, float& b, float& c, float& d) {
    asm volatile("s_nop 1\n\t"
                 "v_add_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %1, %1, %1 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %2, %2, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %3, %3, %3 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %1, %1, %1 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %2, %2, %2 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %3, %3, %3 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %1, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %2, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %3, %3, %3 row_half_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %1, %1, %1 row_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %2, %2, %2 row_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %3, %3, %3 row_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
}
__device__ __forceinline__ void row16_sum2(float& a, float& b) {
    asm volatile("s_nop 1\n\t"
                 "v_add_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %1, %1, %1 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "s_nop 0\n\t"
                 "v_add_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %1, %1, %1 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "s_nop 0\n\t"
                 "v_add_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %1, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "s_nop 0\n\t"
                 "v_add_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "v_add_f32_dpp %1, %1, %1 row_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void row16_sum1(float& a) {
    asm volatile("s_nop 1\n\t"
                 "v_add_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "s_nop 1\n\t"
                 "v_add_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "s_nop 1\n\t"
                 "v_add_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 "s_nop 1\n\t"
                 "v_add_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                 : "+v"(a));
}
template <int N>
__device__ __forceinline__ void row16_sum_n(float (&x)[N]) {
#pragma unroll
    for (int i = 0; i + 3 < N; i += 4) row16_sum4(x[i], x[i + 1], x[i + 2], x[i + 3]);
    if constexpr (N % 4 >= 2) row16_sum2(x[N - (N % 4)], x[N - (N % 4) + 1]);
    if constexpr (N % 2 == 1) row16_sum1(x[N - 1]);
}

// ---------------------------------------------------------------------------
// knot span and basis
// ---------------------------------------------------------------------------

// Clamp a parameter into the domain [U_deg, U_{n+1}] (n+1 = control points).
__device__ __forceinline__ float clamp_param(const float* __restrict__ U, int deg, int n, float x) {
    return fminf(fmaxf(x, U[deg]), U[n + 1]);
}

// Half-open span: the k in [deg, n] with U_k <= x < U_{k+1}; x == U_{n+1}
// gives n.  Binary search over float comparisons, so the result is exact.
__device__ __forceinline__ int find_span(const float* __restrict__ U, int deg, int n, float x) {
    if (x >= U[n + 1]) return n;
    int lo = deg, hi = n + 1;  // invariant: U[lo] <= x < U[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (U[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Reverse-mode derivative of Phi = sum_r e[r] N_{k-D+r}^D(x) with respect to
// the knots U_{k-D} .. U_{k+D+1} (gU[t] <-> U_{k-D+t}), through the
// recursion N_i^d = alpha N_i^{d-1} + beta N_{i+1}^{d-1},
// alpha = (x-U_i)/(U_{i+d}-U_i), beta = (U_{i+d+1}-x)/(U_{i+d+1}-U_{i+1}).
// The degree-0 indicator contributes no knot derivative (zero-bandwidth
// limit of the paper's smoothing), so only the alpha/beta factors do.
// FP32: every factor is a ratio of FP32 knot differences, taken as a product
// with the hardware reciprocal refined by one Newton step, so each term is
// accurate to a few ulp.
template <int D>
__device__ __forceinline__ void basis_knot_adjoint(const float* __restrict__ U, int k, float x,
                                                   const float e[D + 1], float gU[2 * D + 2]) {
    // forward triangle T[d][idx] = N_{k-d+idx}^d, with the reciprocals of the
    // alpha / beta denominators kept for the reverse sweep (0 for an empty
    // knot interval: the term is dropped)
    float T[D + 1][D + 1];
    float ia[D + 1][D + 1], ib[D + 1][D + 1];
    T[0][0] = 1.0f;
#pragma unroll
    for (int d = 1; d <= D; ++d) {
#pragma unroll
        for (int idx = 0; idx <= d; ++idx) {
            const int i = k - d + idx;
            float v = 0.0f;
            ia[d][idx] = ib[d][idx] = 0.0f;
            if (idx >= 1) {
                const float den = U[i + d] - U[i];
                if (den != 0.0f) {
                    ia[d][idx] = recip(den);
                    v += (x - U[i]) * ia[d][idx] * T[d - 1][idx - 1];
                }
            }
            if (idx <= d - 1) {
                const float den = U[i + d + 1] - U[i + 1];
                if (den != 0.0f) {
                    ib[d][idx] = recip(den);
                    v += (U[i + d + 1] - x) * ib[d][idx] * T[d - 1][idx];
                }
            }
            T[d][idx] = v;
        }
    }
#pragma unroll
    for (int t = 0; t < 2 * D + 2; ++t) gU[t] = 0.0f;
    float A[D + 1];
#pragma unroll
    for (int r = 0; r <= D; ++r) A[r] = e[r];
#pragma unroll
    for (int d = D; d >= 1; --d) {
        float An[D + 1];
#pragma unroll
        for (int r = 0; r <= D; ++r) An[r] = 0.0f;
#pragma unroll
        for (int idx = 0; idx <= d; ++idx) {
            const int i = k - d + idx;
            const int t = D - d + idx;  // window slot of U_i
            const float Ai = A[idx];
            if (idx >= 1) {
                const float inv = ia[d][idx];
                const float Ui = U[i], Uid = U[i + d];
                const float c = Ai * T[d - 1][idx - 1] * inv * inv;
                An[idx - 1] += Ai * (x - Ui) * inv;
                gU[t] += c * (x - Uid);
                gU[t + d] -= c * (x - Ui);
            }
            if (idx <= d - 1) {
                const float inv = ib[d][idx];
                const float Ui1 = U[i + 1], Uid1 = U[i + d + 1];
                const float c = Ai * T[d - 1][idx] * inv * inv;
                An[idx] += Ai * (Uid1 - x) * inv;
                gU[t + 1] += c * (Uid1 - x);
                gU[t + d + 1] += c * (x - Ui1);
            }
        }
#pragma unroll
        for (int r = 0; r <= D; ++r) A[r] = An[r];
    }
}

// ---------------------------------------------------------------------------
// one surface's arrays
// ---------------------------------------------------------------------------
struct Surf {
    const float* __restrict__ ctrl;  // [nu_c][nv_c][3]
    const float* __restrict__ w;     // [nu_c][nv_c]
    const float* __restrict__ ku;    // [nu_c+p+1]
    const float* __restrict__ kv;    // [nv_c+q+1]
    const float* __restrict__ us;    // [nu_s]
    const float* __restrict__ vs;    // [nv_s]
    int nu_c, nv_c, nu_s, nv_s;
    // Fixed-knot tables (read only by kernels built for them): the span of
    // every sample and its basis row, [nu_s] and [nu_s][p+1] (v likewise).
    const int* __restrict__ tsu;
    const float* __restrict__ tbu;
    const int* __restrict__ tsv;
    const float* __restrict__ tbv;
};

// homogeneous control point Pw_ij = (w x, w y, w z, w)
__device__ __forceinline__ float4 load_pw(const Surf& s, int i, int j) {
    const int ij = i * s.nv_c + j;
    const float* c = s.ctrl + 3 * ij;
    const float wt = s.w[ij];
    return make_float4(c[0] * wt, c[1] * wt, c[2] * wt, wt);
}

// Three consecutive floats as one 12-byte store (global_store_dwordx3): a
// wave writes a row's 64 points as 768 contiguous bytes with one instruction
// instead of three strided ones.  Points are only 4-byte aligned.
typedef float float3u __attribute__((ext_vector_type(3))) __attribute__((aligned(4)));
__device__ __forceinline__ void store3(float* p, float x, float y, float z) {
    float3u v = {x, y, z};
    *reinterpret_cast<float3u*>(p) = v;
}

__device__ __forceinline__ float4 fma4(float a, float4 x, float4 y) {
    return make_float4(__builtin_fmaf(a, x.x, y.x), __builtin_fmaf(a, x.y, y.y),
                       __builtin_fmaf(a, x.z, y.z), __builtin_fmaf(a, x.w, y.w));
}
__device__ __forceinline__ float dot4(float4 a, float4 b) {
    return __builtin_fmaf(a.x, b.x, __builtin_fmaf(a.y, b.y, __builtin_fmaf(a.z, b.z, a.w * b.w)));
}

// R_i(b) = sum_h Nv_h(v_b) Pw[i][jb + h]: control row i contracted along v
// for this lane's sample column (jb = span_v - q).  q <= QM is uniform.
template <int QM>
__device__ __forceinline__ float4 row_contract(const Surf& s, int i, int jb, const float Nv[QM + 1], int q) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int h = 0; h <= QM; ++h)
        if (h <= q) acc = fma4(Nv[h], load_pw(s, i, jb + h), acc);
    return acc;
}

// The D+1 non-zero basis functions N_{k-D..k}^D(x) on span k, by the
// triangular Cox-de Boor scheme with left/right knot distances.  Every
// denominator is a knot difference that contains [U_k, U_{k+1}], so it is
// positive on a non-empty span.  FP32: the differences of FP32 inputs carry
// one rounding each and the divides are reciprocal products, so the values
// are accurate to a few ulp per degree.
template <int D>
__device__ __forceinline__ void basis_f32(const float* __restrict__ U, int k, float x, float N[D + 1]) {
    float left[D + 1], right[D + 1];
    N[0] = 1.0f;
#pragma unroll
    for (int j = 1; j <= D; ++j) {
        left[j] = x - U[k + 1 - j];
        right[j] = U[k + j] - x;
        float saved = 0.0f;
#pragma unroll
        for (int r = 0; r < j; ++r) {
            const float tmp = N[r] * recip(right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
}

// Span and FP32 basis of one sample along a direction with degree D.
template <int D>
__device__ __forceinline__ int sample_basis(const float* __restrict__ U, int nc, float x, float N[D + 1]) {
    const int n = nc - 1;
    const float xc = clamp_param(U, D, n, x);
    const int k = find_span(U, D, n, xc);
    basis_f32<D>(U, k, xc, N);
    return k;
}

// The D+1 non-zero basis functions on span k and their first derivatives in
// x (Appendix A, eq. NURBSuDerivative1 needs dN/du):
//   dN_i^D = D N_i^{D-1} / (U_{i+D} - U_i) - D N_{i+1}^{D-1} / (U_{i+D+1} - U_{i+1}),
// from the degree D-1 functions of the same span.  Each denominator contains
// [U_k, U_{k+1}], so it is positive on a non-empty span.
template <int D>
__device__ __forceinline__ void basis_d1_f32(const float* __restrict__ U, int k, float x, float N[D + 1],
                                             float dN[D + 1]) {
    float Nm[D];
    basis_f32<D - 1>(U, k, x, Nm);  // N_{k-D+1..k}^{D-1}
#pragma unroll
    for (int r = 0; r <= D; ++r) {
        const int i = k - D + r;
        float d = 0.0f;
        if (r >= 1) d += Nm[r - 1] * recip(U[i + D] - U[i]);
        if (r <= D - 1) d -= Nm[r] * recip(U[i + D + 1] - U[i + 1]);
        dN[r] = (float)D * d;
    }
    basis_f32<D>(U, k, x, N);
}

// Span, basis and first derivatives of one sample along a direction.
template <int D>
__device__ __forceinline__ int sample_basis_d1(const float* __restrict__ U, int nc, float x, float N[D + 1],
                                               float dN[D + 1]) {
    const int n = nc - 1;
    const float xc = clamp_param(U, D, n, x);
    const int k = find_span(U, D, n, xc);
    basis_d1_f32<D>(U, k, xc, N, dN);
    return k;
}

// The same with a uniform runtime degree d <= DM; N[d+1..DM] are set to 0.
template <int DM>
__device__ __forceinline__ int sample_basis_rt(const float* __restrict__ U, int nc, float x, int d, float N[DM + 1]) {
#pragma unroll
    for (int r = 0; r <= DM; ++r) N[r] = 0.f;
    int k = 0;
    switch (d) {
#define ND_SB(D)                                                      \
    case D:                                                           \
        if constexpr (D <= DM) {                                      \
            float t[D + 1];                                           \
            k = sample_basis<D>(U, nc, x, t);                         \
            _Pragma("unroll") for (int r = 0; r <= D; ++r) N[r] = t[r]; \
        }                                                             \
        break;
        ND_SB(1) ND_SB(2) ND_SB(3) ND_SB(4) ND_SB(5) ND_SB(6) ND_SB(7)
#undef ND_SB
        default: break;
    }
    return k;
}

}  // namespace nd
