// Chamfer and Hausdorff distances between point sets on gfx950 (the losses
// of NURBS-Diff Sec. 4, eqs. ChamferDistance and HausdorffDistance):
//
//   CD = sum_i min_j |P_i - Q_j| + sum_j min_i |P_i - Q_j|
//   HD = max_i min_j |P_i - Q_j| + max_j min_i |P_i - Q_j|
//
// Which point is nearest (and which distance is largest) is an integer
// decision.  It is taken in float32 on the float32 inputs with the squared
// distance formed as  d2 = fma(dz, dz, fma(dy, dy, dx * dx))  (dz = 0 in the
// plane), a strictly smaller d2 winning, so the first index wins ties; the
// largest d2 with the first index wins for the Hausdorff terms.  Distances,
// sums and gradients are then taken from the chosen pairs: distances in
// FP64, gradients as FP32 unit vectors.
//
// Nearest neighbours (k_nn): brute force.  A workgroup takes 4 x 256 query
// points (4 per lane, in registers) and one contiguous range of the target
// set, staged through LDS 256 points at a time; every lane scans the
// targets in increasing index order.  For small query sets the target set
// is split into ranges over more workgroups, and k_nn_merge keeps, per
// query, the first range with the strictly smallest d2 -- the same result
// as one scan in index order.  Per query-target pair the work is 3
// subtractions, 1 multiply, 2 FMAs, 1 compare and 2 selects: VALU bound.
//
// Gradient with respect to P (k_cd_scatter, k_cd_grad):
//   dCD/dP_i = (P_i - Q_a(i))/|.| + sum_{j : b(j) = i} (P_i - Q_j)/|.|
//   dHD/dP_i = [i = i*] (P_i - Q_a(i*))/|.| + [i = b(j*)] (P_i - Q_j*)/|.|
// (a: nearest target of each point, b: nearest point of each target,
// i*, j* the farthest ones).  The sum over the targets that chose a point
// is accumulated in 2^-40 fixed point with 64-bit integer atomics: exact
// and order-independent, so bitwise reproducible (no float atomics).
#include "device.hpp"
#include "launch.hpp"
#include "../../include/nurbsdiff.h"

#include <algorithm>

namespace nd {
namespace {

constexpr int kNnPerLane = 4;
constexpr int kNnQueries = kWG * kNnPerLane;  // query points per workgroup
constexpr int kNnTile = kWG;                  // targets per LDS stage

__device__ __forceinline__ float nn_d2(float px, float py, float pz, float4 q) {
    const float dx = px - q.x, dy = py - q.y, dz = pz - q.z;
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __fmul_rn(dx, dx)));
}

template <int DIM>
__device__ __forceinline__ float4 load_pt(const float* __restrict__ X, long long i) {
    const float* p = X + i * DIM;
    return make_float4(p[0], p[1], DIM == 3 ? p[2] : 0.f, 0.f);
}

// For each query point X[b][i] the first index of its nearest point in
// Y[b][j0 .. j1) and that squared distance.  Grid: (query blocks, ranges, B).
template <int DIM>
__global__ void __launch_bounds__(kWG) k_nn(const float* __restrict__ X, int n, const float* __restrict__ Y, int m,
                                           int range, int* __restrict__ idx, float* __restrict__ d2, long long stride) {
    __shared__ float4 tile[kNnTile];
    const int b = blockIdx.z;
    const int i0 = blockIdx.x * kNnQueries;
    const int j0 = blockIdx.y * range, j1 = min(m, j0 + range);
    const float* Xb = X + (long long)b * n * DIM;
    const float* Yb = Y + (long long)b * m * DIM;
    float px[kNnPerLane], py[kNnPerLane], pz[kNnPerLane], best[kNnPerLane];
    int bi[kNnPerLane];
#pragma unroll
    for (int r = 0; r < kNnPerLane; ++r) {
        const int i = i0 + r * kWG + (int)threadIdx.x;
        const float4 p = i < n ? load_pt<DIM>(Xb, i) : make_float4(0.f, 0.f, 0.f, 0.f);
        px[r] = p.x;
        py[r] = p.y;
        pz[r] = p.z;
        best[r] = __builtin_inff();
        bi[r] = -1;
    }
    for (int t0 = j0; t0 < j1; t0 += kNnTile) {
        const int cnt = min(kNnTile, j1 - t0);
        __syncthreads();
        if ((int)threadIdx.x < cnt) tile[threadIdx.x] = load_pt<DIM>(Yb, t0 + threadIdx.x);
        __syncthreads();
        if (cnt == kNnTile) {
#pragma unroll 4
            for (int j = 0; j < kNnTile; ++j) {
                const float4 q = tile[j];
#pragma unroll
                for (int r = 0; r < kNnPerLane; ++r) {
                    const float d = nn_d2(px[r], py[r], pz[r], q);
                    if (d < best[r]) {
                        best[r] = d;
                        bi[r] = t0 + j;
                    }
                }
            }
        } else {
            for (int j = 0; j < cnt; ++j) {
                const float4 q = tile[j];
#pragma unroll
                for (int r = 0; r < kNnPerLane; ++r) {
                    const float d = nn_d2(px[r], py[r], pz[r], q);
                    if (d < best[r]) {
                        best[r] = d;
                        bi[r] = t0 + j;
                    }
                }
            }
        }
    }
    // no distance below +inf (or only NaN) in the range: its first target,
    // as an ordered scan that starts from the first target would keep
    const long long o = (long long)b * stride + (long long)blockIdx.y * n;
#pragma unroll
    for (int r = 0; r < kNnPerLane; ++r) {
        const int i = i0 + r * kWG + (int)threadIdx.x;
        if (i < n) {
            const bool none = bi[r] < 0;
            idx[o + i] = none ? j0 : bi[r];
            d2[o + i] = none ? nn_d2(px[r], py[r], pz[r], load_pt<DIM>(Yb, j0)) : best[r];
        }
    }
}

// Per query, the first range whose d2 is strictly smallest (ranges in index
// order, so ties go to the smaller target index, as in one ordered scan).
__global__ void __launch_bounds__(kWG) k_nn_merge(const int* __restrict__ pidx, const float* __restrict__ pd2,
                                                 int n, int nranges, long long stride, int B,
                                                 int* __restrict__ idx, float* __restrict__ d2) {
    const long long t = (long long)blockIdx.x * kWG + threadIdx.x;
    if (t >= (long long)B * n) return;
    const int b = (int)(t / n), i = (int)(t - (long long)b * n);
    const long long o = (long long)b * stride + i;
    float best = pd2[o];
    int bi = pidx[o];
    // eight ranges' partials loaded together, then compared in range order
    constexpr int kU = 8;
    int r = 1;
    for (; r + kU <= nranges; r += kU) {
        float d[kU];
        int ix[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            d[u] = pd2[o + (long long)(r + u) * n];
            ix[u] = pidx[o + (long long)(r + u) * n];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (d[u] < best) {
                best = d[u];
                bi = ix[u];
            }
    }
    for (; r < nranges; ++r) {
        const float d = pd2[o + (long long)r * n];
        if (d < best) {
            best = d;
            bi = pidx[o + (long long)r * n];
        }
    }
    idx[t] = bi;
    d2[t] = best;
}

// FP64 distance of a chosen pair and the FP32 unit vector from Y to X.
template <int DIM>
__device__ __forceinline__ double pair_dist(const float* X, long long i, const float* Y, long long j, float dir[3]) {
    double s = 0.0, d[3];
#pragma unroll
    for (int x = 0; x < DIM; ++x) {
        d[x] = (double)X[i * DIM + x] - (double)Y[j * DIM + x];
        s += d[x] * d[x];
    }
    const double r = sqrt(s);
#pragma unroll
    for (int x = 0; x < 3; ++x) dir[x] = (x < DIM && r > 0.0) ? (float)(d[x] / r) : 0.f;
    return r;
}

// Per cloud pair: the Chamfer sum (FP64) and the Hausdorff arg-maxes.
// k_cd_partial: workgroup k of a pair reduces the points i = k*256 + t +
// c*nblk*256 of P and j likewise of Q (a tree over the workgroup); then
// k_cd_final adds the nblk partials in order.  The arg-maxes take the
// largest float32 d2 with the smallest index.  Fixed order throughout.
struct ChState {
    double cd;
    int istar, jstar;
};
struct ChPart {
    double cd;
    float vi, vj;
    int ii, jj;
};

__device__ __forceinline__ void argmax_merge(float& v, int& i, float v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

template <int DIM>
__global__ void __launch_bounds__(kWG) k_cd_partial(const float* __restrict__ P, int n, const float* __restrict__ Q,
                                                   int m, const int* __restrict__ a, const float* __restrict__ da,
                                                   const int* __restrict__ bq, const float* __restrict__ db,
                                                   ChPart* __restrict__ part) {
    __shared__ double sd[kWG];
    __shared__ float svi[kWG], svj[kWG];
    __shared__ int sii[kWG], sjj[kWG];
    const int k = blockIdx.x, nblk = gridDim.x, b = blockIdx.y, t = threadIdx.x;
    const float* Pb = P + (long long)b * n * DIM;
    const float* Qb = Q + (long long)b * m * DIM;
    const int* ab = a + (long long)b * n;
    const int* bb = bq + (long long)b * m;
    const float* dab = da + (long long)b * n;
    const float* dbb = db + (long long)b * m;
    float dir[3];
    double acc = 0.0;
    float vi = -1.f, vj = -1.f;
    int ii = n, jj = m;
    for (int i = k * kWG + t; i < n; i += nblk * kWG) {
        acc += pair_dist<DIM>(Pb, i, Qb, ab[i], dir);
        argmax_merge(vi, ii, dab[i], i);
    }
    for (int j = k * kWG + t; j < m; j += nblk * kWG) {
        acc += pair_dist<DIM>(Pb, bb[j], Qb, j, dir);
        argmax_merge(vj, jj, dbb[j], j);
    }
    sd[t] = acc;
    svi[t] = vi;
    sii[t] = ii;
    svj[t] = vj;
    sjj[t] = jj;
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if (t < h) {
            sd[t] += sd[t + h];
            argmax_merge(svi[t], sii[t], svi[t + h], sii[t + h]);
            argmax_merge(svj[t], sjj[t], svj[t + h], sjj[t + h]);
        }
        __syncthreads();
    }
    if (t == 0) {
        ChPart o;
        o.cd = sd[0];
        o.vi = svi[0];
        o.ii = sii[0];
        o.vj = svj[0];
        o.jj = sjj[0];
        part[(long long)b * nblk + k] = o;
    }
}

template <int DIM>
__global__ void k_cd_final(const float* __restrict__ P, int n, const float* __restrict__ Q, int m,
                           const int* __restrict__ a, const int* __restrict__ bq, const ChPart* __restrict__ part,
                           int nblk, int B, float* __restrict__ out, ChState* __restrict__ st) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const ChPart* pb = part + (long long)b * nblk;
    double cd = 0.0;
    float vi = -1.f, vj = -1.f;
    int ii = n, jj = m;
    for (int k = 0; k < nblk; ++k) {
        cd += pb[k].cd;
        argmax_merge(vi, ii, pb[k].vi, pb[k].ii);
        argmax_merge(vj, jj, pb[k].vj, pb[k].jj);
    }
    const float* Pb = P + (long long)b * n * DIM;
    const float* Qb = Q + (long long)b * m * DIM;
    float dir[3];
    const double hd = pair_dist<DIM>(Pb, ii, Qb, a[(long long)b * n + ii], dir) +
                      pair_dist<DIM>(Pb, bq[(long long)b * m + jj], Qb, jj, dir);
    out[2 * b] = (float)cd;
    out[2 * b + 1] = (float)hd;
    st[b].cd = cd;
    st[b].istar = ii;
    st[b].jstar = jj;
}

// Fixed-point accumulation of the targets' pulls: each unit vector
// component (|u| <= 1) is rounded to a multiple of 2^-40 and added as a
// 64-bit integer.  Integer addition is exact and associative, so the sums
// do not depend on the order the atomics land in (bitwise reproducible);
// with at most 2^22 targets they stay below 2^62.
constexpr double kFixScale = 1099511627776.0;  // 2^40

template <int DIM>
__global__ void __launch_bounds__(kWG) k_cd_scatter(const float* __restrict__ P, int n, const float* __restrict__ Q,
                                                   int m, const int* __restrict__ bq,
                                                   unsigned long long* __restrict__ acc) {
    const int b = blockIdx.y;
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= m) return;
    const float* Pb = P + (long long)b * n * DIM;
    const float* Qb = Q + (long long)b * m * DIM;
    const int i = bq[(long long)b * m + j];
    double d[3], s = 0.0;
#pragma unroll
    for (int x = 0; x < DIM; ++x) {
        d[x] = (double)Pb[(long long)i * DIM + x] - (double)Qb[(long long)j * DIM + x];
        s += d[x] * d[x];
    }
    const double r = sqrt(s);
    if (r == 0.0) return;
    unsigned long long* o = acc + ((long long)b * n + i) * 3;
#pragma unroll
    for (int x = 0; x < DIM; ++x)
        atomicAdd(o + x, (unsigned long long)__double2ll_rn(d[x] / r * kFixScale));
}

// dCD/dP and dHD/dP, one thread per point of P.
template <int DIM>
__global__ void __launch_bounds__(kWG) k_cd_grad(const float* __restrict__ P, int n, const float* __restrict__ Q,
                                                int m, const int* __restrict__ a, const int* __restrict__ bq,
                                                const ChState* __restrict__ st,
                                                const unsigned long long* __restrict__ acc, float* __restrict__ gcd,
                                                float* __restrict__ ghd) {
    const int b = blockIdx.y;
    const int i = blockIdx.x * kWG + threadIdx.x;
    if (i >= n) return;
    const float* Pb = P + (long long)b * n * DIM;
    const float* Qb = Q + (long long)b * m * DIM;
    const int ai = a[(long long)b * n + i];
    double d[3] = {0.0, 0.0, 0.0}, s = 0.0;
#pragma unroll
    for (int x = 0; x < DIM; ++x) {
        d[x] = (double)Pb[(long long)i * DIM + x] - (double)Qb[(long long)ai * DIM + x];
        s += d[x] * d[x];
    }
    const double r = sqrt(s);
    double u[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) u[x] = r > 0.0 ? d[x] / r : 0.0;
    const long long o = ((long long)b * n + i) * DIM;
    if (gcd) {
        const unsigned long long* ac = acc + ((long long)b * n + i) * 3;
#pragma unroll
        for (int x = 0; x < DIM; ++x) gcd[o + x] = (float)(u[x] + (double)(long long)ac[x] / kFixScale);
    }
    if (ghd) {
        const ChState cs = st[b];
        double h[3] = {0.0, 0.0, 0.0};
        if (i == cs.istar) {
#pragma unroll
            for (int x = 0; x < 3; ++x) h[x] += u[x];
        }
        if (i == bq[(long long)b * m + cs.jstar]) {
            double e[3], s2 = 0.0;
#pragma unroll
            for (int x = 0; x < DIM; ++x) {
                e[x] = (double)Pb[(long long)i * DIM + x] - (double)Qb[(long long)cs.jstar * DIM + x];
                s2 += e[x] * e[x];
            }
            const double r2 = sqrt(s2);
#pragma unroll
            for (int x = 0; x < DIM; ++x) h[x] += r2 > 0.0 ? e[x] / r2 : 0.0;
        }
#pragma unroll
        for (int x = 0; x < DIM; ++x) ghd[o + x] = (float)h[x];
    }
}

template <int DIM>
hipError_t nn_launch(hipStream_t st, int B, const float* X, int n, const float* Y, int m, const NnSplit& sp,
                     int* idx, float* d2, int* pidx, float* pd2) {
    const dim3 grid((unsigned)((n + kNnQueries - 1) / kNnQueries), (unsigned)sp.nranges, (unsigned)B);
    if (sp.nranges == 1) {
        hipLaunchKernelGGL((k_nn<DIM>), grid, dim3(kWG), 0, st, X, n, Y, m, sp.range, idx, d2, (long long)n);
        return hipGetLastError();
    }
    const long long stride = (long long)sp.nranges * n;
    hipLaunchKernelGGL((k_nn<DIM>), grid, dim3(kWG), 0, st, X, n, Y, m, sp.range, pidx, pd2, stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long items = (long long)B * n;
    hipLaunchKernelGGL(k_nn_merge, dim3((unsigned)((items + kWG - 1) / kWG)), dim3(kWG), 0, st, pidx, pd2, n,
                       sp.nranges, stride, B, idx, d2);
    return hipGetLastError();
}

}  // namespace

NnSplit nn_split(int B, int n, int m, int num_cus) {
    NnSplit s;
    const long long qblocks = (long long)B * ((n + kNnQueries - 1) / kNnQueries);
    const long long want = 4ll * std::max(num_cus, 1);  // workgroups to fill the chip a few times over
    const int max_ranges = std::max(1, (m + kNnTile - 1) / kNnTile);
    long long r = qblocks >= want ? 1 : (want + qblocks - 1) / qblocks;
    s.nranges = (int)std::min<long long>(r, max_ranges);
    const int tiles = (m + kNnTile - 1) / kNnTile;
    const int tiles_per = (tiles + s.nranges - 1) / s.nranges;
    s.range = std::max(1, tiles_per) * kNnTile;
    s.nranges = std::max(1, (m + s.range - 1) / s.range);
    return s;
}

hipError_t launch_nn(int dim, hipStream_t st, int B, const float* X, int n, const float* Y, int m,
                     const NnSplit& sp, int* idx, float* d2, int* pidx, float* pd2) {
    if (dim == 3) return nn_launch<3>(st, B, X, n, Y, m, sp, idx, d2, pidx, pd2);
    if (dim == 2) return nn_launch<2>(st, B, X, n, Y, m, sp, idx, d2, pidx, pd2);
    return hipErrorInvalidValue;
}

int cd_partials(int n, int m) { return std::max(1, std::min(256, (n + m + 2047) / 2048)); }

hipError_t launch_cd(int dim, hipStream_t st, int B, const float* P, int n, const float* Q, int m, const int* a,
                     const float* da, const int* bq, const float* db, float* out, void* state, void* part,
                     void* acc, float* gcd, float* ghd) {
    ChState* cs = reinterpret_cast<ChState*>(state);
    ChPart* cp = reinterpret_cast<ChPart*>(part);
    unsigned long long* ac = reinterpret_cast<unsigned long long*>(acc);
    const int nblk = cd_partials(n, m);
    const dim3 gp((unsigned)nblk, (unsigned)B), gf((unsigned)((B + kWG - 1) / kWG));
    const dim3 gn((unsigned)((n + kWG - 1) / kWG), (unsigned)B), gm((unsigned)((m + kWG - 1) / kWG), (unsigned)B);
    const bool grads = gcd || ghd;
#define ND_CD(D)                                                                                               \
    hipLaunchKernelGGL((k_cd_partial<D>), gp, dim3(kWG), 0, st, P, n, Q, m, a, da, bq, db, cp);                \
    hipLaunchKernelGGL((k_cd_final<D>), gf, dim3(kWG), 0, st, P, n, Q, m, a, bq, cp, nblk, B, out, cs);        \
    if (gcd) {                                                                                                 \
        hipError_t z = launch_zero(st, reinterpret_cast<float*>(ac), (size_t)B * n * 3 * 2);                   \
        if (z != hipSuccess) return z;                                                                         \
        hipLaunchKernelGGL((k_cd_scatter<D>), gm, dim3(kWG), 0, st, P, n, Q, m, bq, ac);                       \
    }                                                                                                          \
    if (grads) hipLaunchKernelGGL((k_cd_grad<D>), gn, dim3(kWG), 0, st, P, n, Q, m, a, bq, cs, ac, gcd, ghd);
    if (dim == 3) { ND_CD(3) }
    else if (dim == 2) { ND_CD(2) }
    else return hipErrorInvalidValue;
#undef ND_CD
    return hipGetLastError();
}

size_t cd_part_bytes(int n, int m) { return sizeof(ChPart) * (size_t)cd_partials(n, m); }

size_t cd_state_bytes() { return sizeof(ChState); }

}  // namespace nd
