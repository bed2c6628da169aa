// Forward, backward and finalize work units for NURBS surfaces on gfx950.
//
// Work decomposition
// ------------------
// A *tile* is (surface, 64 consecutive sample columns, a range of sample
// rows) and is processed by one wave64: lane l owns sample column
// b = col0 + l for every row of the range.  Each lane keeps its column's
// span and q+1 basis values in registers for the whole tile.
//
// Forward (Sec. 3.1.2 of NURBS-Diff; Alg. Forward over all points):
//   S'(a,b) = sum_r Nu_r(a) R_{ka-p+r}(b),  R_i(b) = sum_h Nv_h(b) Pw[i][kb-q+h]
// The p+1 rows R_i that the current u-span touches live in registers as a
// sliding window; the window advances when the row span advances, so each
// row is contracted along v once per tile, not once per point.  The
// per-point work is 4(p+1) FMAs, the rational divide and a 12-byte store.
//
// Backward (Sec. 3.2, Alg. Backward as a vector-Jacobian product): per point
//   h = dL/dS' = (g / W, -(g . S) / W)         (eqs. NURBSuDerivative4/5)
//   G_i(b) += Nu_r(a) h   for the window rows   -> dL/dPw after the v-sum
//   E_r(a) = sum_b R_i(b) . h = dL/dNu_r(a)     (eq. NURBSvDerivative6)
// When a control row leaves the window its accumulator G_i(b) is final for
// the tile and is *flushed*: (i) f_h(b) += Pw[i][kb-q+h] . G_i(b) builds
// dL/dNv_h(b); (ii) the q+1 products Nv_h(b) G_i(b) are summed over the
// lanes that share a v-span by a segmented scan, and one lane per control
// column writes the tile's partial dL/dPw row.  No atomics: each value is
// written once to a tile-indexed workspace slot, and the finalize pass adds
// slots in a fixed order, so results are bitwise reproducible and do not
// depend on which wave ran which tile.
//
// Finalize, one workgroup per surface: dL/dPw = sum of tile rectangles;
// dL/dP = w dL/dPw_xyz, dL/dw = P . dL/dPw_xyz + dL/dPw_w; dL/dU_k by the
// reverse-mode knot derivative of each row's basis weighted with e(a)
// (Sec. 3.2.1), dL/dV_k likewise with f(b).
#pragma once
#include "device.hpp"

namespace nd {

// --------------------------------------------------------------------------
// workspace layout of one backward tile (bytes from the slot start):
//   [0, 16)                      int4 header {i0, i1, j0, j1}
//   [16, 16 + 16*rect_cap)       float4 rect [(i1-i0+1)][(j1-j0+1)]
//   then float e[rows][P+1], then float f[64][Q+1]
// --------------------------------------------------------------------------
struct SlotView {
    int* hdr;
    float4* rect;
    float* e;
    float* f;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline size_t slot_bytes(int p, int q, int nu_c, int nv_c, int rows) {
    size_t b = 16 + 16 * (size_t)nu_c * nv_c;
    b += align16(sizeof(float) * (size_t)rows * (p + 1));
    b += align16(sizeof(float) * (size_t)kWave * (q + 1));
    return b;
}

__device__ __forceinline__ SlotView slot_view(char* base, int p, int nu_c, int nv_c, int rows) {
    SlotView v;
    v.hdr = reinterpret_cast<int*>(base);
    v.rect = reinterpret_cast<float4*>(base + 16);
    char* e = base + 16 + 16 * (size_t)nu_c * nv_c;
    v.e = reinterpret_cast<float*>(e);
    v.f = reinterpret_cast<float*>(e + align16(sizeof(float) * (size_t)rows * (p + 1)));
    return v;
}

// per-wave LDS scratch of the backward tile
struct BwdLds {
    float4 col[kWave * (kMaxDeg + 1)];  // segment sums, [head lane][h]
    int head_of[kWG];                   // key offset -> head lane, or -1
};

// device error word (first error wins)
__device__ __forceinline__ void post_error(int* err, int code) {
    if (err) atomicCAS(err, 0, code);
}

// Data checks of one surface (NURBS_VALIDATE), done by the wave that owns
// the surface's first tile.
__device__ __forceinline__ void validate_surface(const Surf& s, int P, int Q, int* err) {
    const int lane = lane_id();
    const int nU = s.nu_c + P + 1, nV = s.nv_c + Q + 1;
    bool bad_k = false, bad_w = false, bad_d = false;
    for (int i = lane; i + 1 < nU; i += kWave) bad_k |= !(s.ku[i] <= s.ku[i + 1]);
    for (int i = lane; i + 1 < nV; i += kWave) bad_k |= !(s.kv[i] <= s.kv[i + 1]);
    if (lane == 0) {
        bad_k |= !(s.ku[P] < s.ku[P + 1]) || !(s.ku[s.nu_c - 1] < s.ku[s.nu_c]);
        bad_k |= !(s.kv[Q] < s.kv[Q + 1]) || !(s.kv[s.nv_c - 1] < s.kv[s.nv_c]);
    }
    for (int i = lane; i < s.nu_c * s.nv_c; i += kWave) bad_w |= !(s.w[i] > 0.f);
    const float ulo = s.ku[P], uhi = s.ku[s.nu_c], vlo = s.kv[Q], vhi = s.kv[s.nv_c];
    for (int a = lane; a < s.nu_s; a += kWave) {
        const float x = s.us[a];
        bad_d |= !(x >= ulo && x <= uhi);
        if (a + 1 < s.nu_s) bad_d |= !(x <= s.us[a + 1]);
    }
    for (int b = lane; b < s.nv_s; b += kWave) {
        const float x = s.vs[b];
        bad_d |= !(x >= vlo && x <= vhi);
        if (b + 1 < s.nv_s) bad_d |= !(x <= s.vs[b + 1]);
    }
    if (__any(bad_k) && lane == 0) post_error(err, -3);
    if (__any(bad_w) && lane == 0) post_error(err, -5);
    if (__any(bad_d) && lane == 0) post_error(err, -4);
}

// --------------------------------------------------------------------------
// forward tile
// --------------------------------------------------------------------------
template <int P, int QM>
__device__ __forceinline__ void fwd_tile(const Surf& s, int q, int col0, int row0, int row1, float* __restrict__ pts) {
    const int lane = lane_id();
    const int b = col0 + lane;
    const bool act = b < s.nv_s;
    float Nv[QM + 1];
    const int kb = sample_basis_rt<QM>(s.kv, s.nv_c, s.vs[act ? b : s.nv_s - 1], q, Nv);
    const int jb = kb - q;

    float4 R[P + 1];
    int cur = -1;  // span of the window (rows cur-P .. cur); -1 = empty
    for (int a0 = row0; a0 < row1; a0 += kWave) {
        const int nr = min(kWave, row1 - a0);
        float Nu_l[P + 1];
        const int ka_l = sample_basis<P>(s.ku, s.nu_c, s.us[a0 + min(lane, nr - 1)], Nu_l);
        for (int t = 0; t < nr; ++t) {
            const int ka = bcast_lane(ka_l, t);
            if (ka != cur) {
                if (cur >= 0 && ka > cur && ka - cur <= P) {
                    do {
#pragma unroll
                        for (int r = 0; r < P; ++r) R[r] = R[r + 1];
                        ++cur;
                        R[P] = row_contract<QM>(s, cur, jb, Nv, q);
                    } while (cur < ka);
                } else {
                    cur = ka;
#pragma unroll
                    for (int r = 0; r <= P; ++r) R[r] = row_contract<QM>(s, ka - P + r, jb, Nv, q);
                }
            }
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int r = 0; r <= P; ++r) acc = fma4(bcast_lane(Nu_l[r], t), R[r], acc);
            const float rw = recip(acc.w);
            if (act) {
                float* o = pts + 3 * ((size_t)(a0 + t) * s.nv_s + b);
                o[0] = acc.x * rw;
                o[1] = acc.y * rw;
                o[2] = acc.z * rw;
            }
        }
    }
}

// --------------------------------------------------------------------------
// backward tile
// --------------------------------------------------------------------------
template <int QM>
struct BwdState {
    float Nv[QM + 1];
    int kb, jb;
    bool act;
    int key_off;      // kb - kfirst for active lanes
    int nkeys;        // distinct keys span kfirst..klast
    int j0, ncols;    // rect column range
    int seg_first;    // first lane of this lane's segment
    int nsteps;       // scan steps needed (max segment length)
    bool head;        // last lane of its segment
    int q;            // degree in v (uniform, <= QM)
    float f[QM + 1];  // dL/dNv_h(v_b) partial
};

// Flush control row i (accumulator G) of the tile: dV partial and the
// rect row i - i0 of dL/dPw.
template <int QM>
__device__ __forceinline__ void flush_row(const Surf& s, BwdState<QM>& st, int i, int i0, float4 G,
                                          float4* __restrict__ rect, BwdLds* L, bool want_pw,
                                          bool want_kv) {
    const int lane = lane_id();
    const int q = st.q;
    if (want_kv) {
#pragma unroll
        for (int h = 0; h <= QM; ++h)
            if (h <= q) st.f[h] += dot4(load_pw(s, i, st.jb + h), G);
    }
    if (!want_pw) return;
    float4 x[QM + 1];
#pragma unroll
    for (int h = 0; h <= QM; ++h) {
        const float c = st.act ? st.Nv[h] : 0.f;
        x[h] = make_float4(c * G.x, c * G.y, c * G.z, c * G.w);
    }
    // segmented inclusive scan over lanes sharing a v-span
    for (int step = 0, d = 1; step < st.nsteps; ++step, d <<= 1) {
        const bool take = (lane - d) >= st.seg_first;
#pragma unroll
        for (int h = 0; h <= QM; ++h) {
            if (h > q) continue;
            float4 y;
            y.x = __shfl_up(x[h].x, d, kWave);
            y.y = __shfl_up(x[h].y, d, kWave);
            y.z = __shfl_up(x[h].z, d, kWave);
            y.w = __shfl_up(x[h].w, d, kWave);
            if (take) {
                x[h].x += y.x;
                x[h].y += y.y;
                x[h].z += y.z;
                x[h].w += y.w;
            }
        }
    }
    if (st.head) {
#pragma unroll
        for (int h = 0; h <= QM; ++h)
            if (h <= q) L->col[lane * (QM + 1) + h] = x[h];
    }
    wave_lds_sync();
    // control column j = j0 + c gathers keys kfirst + c - h
    for (int c = lane; c < st.ncols; c += kWave) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int h = 0; h <= QM; ++h) {
            const int o = c - h;
            const int hl = (h <= q && o >= 0 && o < st.nkeys) ? L->head_of[o] : -1;
            if (hl >= 0) {
                const float4 v = L->col[hl * (QM + 1) + h];
                acc.x += v.x;
                acc.y += v.y;
                acc.z += v.z;
                acc.w += v.w;
            }
        }
        rect[(size_t)(i - i0) * st.ncols + c] = acc;
    }
    wave_lds_sync();
}

// Column set-up of a backward tile (independent of the degree in u): the
// lane's v-span and basis, and the segment structure of the spans.
template <int QM>
__device__ __forceinline__ void bwd_columns(const Surf& s, int q, int col0, BwdState<QM>& st, BwdLds* L) {
    const int lane = lane_id();
    st.q = q;
    const int b = col0 + lane;
    st.act = b < s.nv_s;
    st.kb = sample_basis_rt<QM>(s.kv, s.nv_c, s.vs[st.act ? b : s.nv_s - 1], q, st.Nv);
    st.jb = st.kb - q;
#pragma unroll
    for (int h = 0; h <= QM; ++h) st.f[h] = 0.f;

    // segment structure of the columns (spans are non-decreasing in b)
    const int nact = min(kWave, s.nv_s - col0);
    const int kfirst = bcast_lane(st.kb, 0);
    const int klast = bcast_lane(st.kb, nact - 1);
    st.nkeys = klast - kfirst + 1;
    st.j0 = kfirst - q;
    st.ncols = klast - st.j0 + 1;
    st.key_off = st.kb - kfirst;
    const int kb_next = __shfl_down(st.kb, 1, kWave);
    st.head = st.act && (lane == nact - 1 || kb_next != st.kb);
    {   // first lane of the segment: max over lanes <= me with a different key, +1
        const int kb_prev = __shfl_up(st.kb, 1, kWave);
        const bool starts = st.act && (lane == 0 || kb_prev != st.kb);
        int f = starts ? lane : 0;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int y = __shfl_up(f, d, kWave);
            if (lane >= d) f = max(f, y);
        }
        st.seg_first = st.act ? f : kWave;  // inactive lanes never take
        int len = st.act ? lane - f + 1 : 1;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) len = max(len, __shfl_xor(len, d, kWave));
        int steps = 0;
        while ((1 << steps) < len) ++steps;
        st.nsteps = steps;
    }
    for (int o = lane; o < st.nkeys; o += kWave) L->head_of[o] = -1;
    wave_lds_sync();
    if (st.head) L->head_of[st.key_off] = lane;
    wave_lds_sync();
}

template <int P, int QM>
__device__ __forceinline__ void bwd_rows(const Surf& s, BwdState<QM>& st, int col0, int row0, int row1,
                         const float* __restrict__ gpts, SlotView out, BwdLds* L, unsigned mask) {
    const int lane = lane_id();
    const bool want_pw = (mask & 3u) != 0;
    const bool want_ku = (mask & 4u) != 0;
    const bool want_kv = (mask & 8u) != 0;
    const int q = st.q;
    const int b = col0 + lane;
    float4 R[P + 1], G[P + 1];
    int cur = -1, i0 = 0;
    // Slide the window until its last row is `target`, flushing every row
    // that leaves it.  Rows past the last control row are never loaded; the
    // end-of-tile drain uses this with target = cur + P + 1.
    auto advance = [&](int target) {
        while (cur < target) {
            flush_row<QM>(s, st, cur - P, i0, G[0], out.rect, L, want_pw, want_kv);
#pragma unroll
            for (int r = 0; r < P; ++r) {
                R[r] = R[r + 1];
                G[r] = G[r + 1];
            }
            ++cur;
            G[P] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (cur < s.nu_c) R[P] = row_contract<QM>(s, cur, st.jb, st.Nv, q);
        }
    };
    for (int a0 = row0; a0 < row1; a0 += kWave) {
        const int nr = min(kWave, row1 - a0);
        float Nu_l[P + 1];
        const int ka_l = sample_basis<P>(s.ku, s.nu_c, s.us[a0 + min(lane, nr - 1)], Nu_l);
        for (int t = 0; t < nr; ++t) {
            const int ka = bcast_lane(ka_l, t);
            if (cur < 0) {
                cur = ka;
                i0 = ka - P;
#pragma unroll
                for (int r = 0; r <= P; ++r) {
                    R[r] = row_contract<QM>(s, ka - P + r, st.jb, st.Nv, q);
                    G[r] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
            } else {
                // rows are non-decreasing, so the window only moves forward
                advance(ka);
            }
            float Nu[P + 1];
#pragma unroll
            for (int r = 0; r <= P; ++r) Nu[r] = bcast_lane(Nu_l[r], t);
            // recompute S' (nothing is saved by the forward)
            float4 sp = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int r = 0; r <= P; ++r) sp = fma4(Nu[r], R[r], sp);
            const float rw = recip(sp.w);
            float gx = 0.f, gy = 0.f, gz = 0.f;
            if (st.act) {
                const float* gp = gpts + 3 * ((size_t)(a0 + t) * s.nv_s + b);
                gx = gp[0];
                gy = gp[1];
                gz = gp[2];
            }
            const float cx = gx * rw, cy = gy * rw, cz = gz * rw;
            const float cw = -(cx * sp.x + cy * sp.y + cz * sp.z) * rw;
            const float4 hv = make_float4(cx, cy, cz, cw);
#pragma unroll
            for (int r = 0; r <= P; ++r) G[r] = fma4(Nu[r], hv, G[r]);
            if (want_ku) {
                float E[P + 1];
#pragma unroll
                for (int r = 0; r <= P; ++r) E[r] = wave_sum(dot4(R[r], hv));
                if (lane <= P) {
                    float v = E[0];
#pragma unroll
                    for (int r = 1; r <= P; ++r) v = (lane == r) ? E[r] : v;
                    out.e[(size_t)(a0 + t - row0) * (P + 1) + lane] = v;
                }
            }
        }
    }
    // flush the rows still in the window
    const int i1 = cur;
    advance(cur + P + 1);
    if (want_kv) {
#pragma unroll
        for (int h = 0; h <= QM; ++h)
            if (h <= q) out.f[lane * (q + 1) + h] = st.f[h];
    }
    if (lane == 0) {
        out.hdr[0] = i0;
        out.hdr[1] = i1;
        out.hdr[2] = st.j0;
        out.hdr[3] = st.j0 + st.ncols - 1;
    }
}

template <int P, int QM>
__device__ __forceinline__ void bwd_tile(const Surf& s, int q, int col0, int row0, int row1,
                         const float* __restrict__ gpts, SlotView out, BwdLds* L, unsigned mask) {
    BwdState<QM> st;
    bwd_columns<QM>(s, q, col0, st, L);
    bwd_rows<P, QM>(s, st, col0, row0, row1, gpts, out, L, mask);
}

// --------------------------------------------------------------------------
// finalize: one workgroup (kWG threads) per surface
// --------------------------------------------------------------------------
struct FinLds {
    double contrib[kWG * (2 * kMaxDeg + 2)];  // per sample, knot-window adjoints
    int span[kWG];                            // span of each sample of the chunk
};

// Tiles of one surface in their fixed summation order: slot pointer,
// column start and row range of tile t.
struct TileRef {
    const char* slot;
    int col0, row0, row1;
    int alloc_rows;  // rows the slot was sized for (>= row1 - row0)
};

// Knot gradient of one direction: for every sample x_a of the direction,
// coef(a)[r] = dL/dN_{k_a-D+r}(x_a) is turned into per-knot adjoints by
// basis_knot_adjoint; the adjoints are then summed over samples in sample
// order (chunks of kWG samples staged in LDS), one thread per knot.
template <int D, class CoefAt>
__device__ __forceinline__ void knot_gradient(const float* __restrict__ U, int nc, const float* __restrict__ xs, int ns,
                              CoefAt coef_at, float* __restrict__ gout, FinLds* L) {
    constexpr int W = 2 * D + 2;
    const int tid = threadIdx.x;
    const int nk = nc + D + 1;
    const int n = nc - 1;
    double acc = 0.0;
    for (int a0 = 0; a0 < ns; a0 += kWG) {
        const int a = a0 + tid;
        int k = -1;
        if (a < ns) {
            const float x = clamp_param(U, D, n, xs[a]);
            k = find_span(U, D, n, x);
            double e[D + 1];
            coef_at(a, e);
            double g[W];
            basis_knot_adjoint<D>(U, k, x, e, g);
#pragma unroll
            for (int t = 0; t < W; ++t) L->contrib[tid * W + t] = g[t];
        }
        L->span[tid] = k;
        __syncthreads();
        const int cnt = min(kWG, ns - a0);
        if (tid < nk) {
            for (int r = 0; r < cnt; ++r) {
                const int t = tid - (L->span[r] - D);
                if (t >= 0 && t < W) acc += L->contrib[r * W + t];
            }
        }
        __syncthreads();
    }
    if (tid < nk) gout[tid] = (float)acc;
}

template <int P, int Q, class TileAt>
__device__ __forceinline__ void finalize_surface(const Surf& s, int ntiles, TileAt tile_at, float* __restrict__ gctrl,
                                 float* __restrict__ gw, float* __restrict__ gku, float* __restrict__ gkv,
                                 unsigned mask, FinLds* L) {
    const int tid = threadIdx.x;
    const size_t rect_bytes = 16 * (size_t)s.nu_c * s.nv_c;
    // dL/dP and dL/dw from the tile rectangles, tiles in fixed order
    if (mask & 3u) {
        for (int ij = tid; ij < s.nu_c * s.nv_c; ij += kWG) {
            const int i = ij / s.nv_c, j = ij - i * s.nv_c;
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int t = 0; t < ntiles; ++t) {
                const TileRef tr = tile_at(t);
                const int* hdr = reinterpret_cast<const int*>(tr.slot);
                const int i0 = hdr[0], i1 = hdr[1], j0 = hdr[2], j1 = hdr[3];
                if (i >= i0 && i <= i1 && j >= j0 && j <= j1) {
                    const float4 v = reinterpret_cast<const float4*>(tr.slot + 16)[(size_t)(i - i0) * (j1 - j0 + 1) + (j - j0)];
                    acc.x += v.x;
                    acc.y += v.y;
                    acc.z += v.z;
                    acc.w += v.w;
                }
            }
            const float wt = s.w[ij];
            const float* pc = s.ctrl + 3 * ij;
            if (mask & 1u) {
                gctrl[3 * ij + 0] = wt * acc.x;
                gctrl[3 * ij + 1] = wt * acc.y;
                gctrl[3 * ij + 2] = wt * acc.z;
            }
            if (mask & 2u) gw[ij] = pc[0] * acc.x + pc[1] * acc.y + pc[2] * acc.z + acc.w;
        }
    }
    // dL/dU: e(a) = sum over the column tiles covering row a
    if (mask & 4u) {
        auto coef = [&](int a, double e[P + 1]) {
#pragma unroll
            for (int r = 0; r <= P; ++r) e[r] = 0.0;
            for (int t = 0; t < ntiles; ++t) {
                const TileRef tr = tile_at(t);
                if (a >= tr.row0 && a < tr.row1) {
                    const float* ev = reinterpret_cast<const float*>(tr.slot + 16 + rect_bytes) +
                                      (size_t)(a - tr.row0) * (P + 1);
#pragma unroll
                    for (int r = 0; r <= P; ++r) e[r] += (double)ev[r];
                }
            }
        };
        knot_gradient<P>(s.ku, s.nu_c, s.us, s.nu_s, coef, gku, L);
    }
    // dL/dV: f(b) = sum over the row tiles covering column b
    if (mask & 8u) {
        auto coef = [&](int b, double f[Q + 1]) {
#pragma unroll
            for (int h = 0; h <= Q; ++h) f[h] = 0.0;
            for (int t = 0; t < ntiles; ++t) {
                const TileRef tr = tile_at(t);
                if (b >= tr.col0 && b < tr.col0 + kWave) {
                    const float* fv = reinterpret_cast<const float*>(
                        tr.slot + 16 + rect_bytes + align16(sizeof(float) * (size_t)tr.alloc_rows * (P + 1)));
#pragma unroll
                    for (int h = 0; h <= Q; ++h) f[h] += (double)fv[(b - tr.col0) * (Q + 1) + h];
                }
            }
        };
        knot_gradient<Q>(s.kv, s.nv_c, s.vs, s.nv_s, coef, gkv, L);
    }
}

}  // namespace nd
