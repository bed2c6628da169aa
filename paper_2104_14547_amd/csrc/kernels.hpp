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
// control-row ring: the rows of the u-window (and the next one) for the
// tile's control columns j0 .. j0+ncols-1, as homogeneous points in LDS
// --------------------------------------------------------------------------
constexpr int kRingCap = 384;  // float4 entries per wave (6 KiB)
constexpr int kEBatch = 16;    // rows per batched reduction of dL/dN(u)

struct Ring {
    float4* base;  // LDS, kRingCap entries
    int j0, ncols, nslots;
    bool on;       // false: the tile's column range does not fit, read Pw from global
};

__device__ __forceinline__ float4* ring_row(const Ring& rg, int i) { return rg.base + (i % rg.nslots) * rg.ncols; }

// Lanes load control row i (columns j0 .. j0+ncols-1) into registers; the
// ring stores them later, so the load latency overlaps other work.
struct RowPrefetch {
    float4 v;  // column j0 + lane (the ring holds at most 64 columns)
};

__device__ __forceinline__ void prefetch_row(const Surf& s, const Ring& rg, int i, RowPrefetch& pf) {
    const int lane = lane_id();
    if (i < s.nu_c && lane < rg.ncols) pf.v = load_pw(s, i, rg.j0 + lane);
}

__device__ __forceinline__ void store_row(const Ring& rg, int i, const RowPrefetch& pf) {
    const int lane = lane_id();
    if (lane < rg.ncols) ring_row(rg, i)[lane] = pf.v;
}

// R_i(b) for this lane's column from the ring (or from global memory).
template <int QM>
__device__ __forceinline__ float4 ring_contract(const Surf& s, const Ring& rg, int i, int jb,
                                                const float Nv[QM + 1], int q) {
    if (!rg.on) return row_contract<QM>(s, i, jb, Nv, q);
    const float4* row = ring_row(rg, i) + (jb - rg.j0);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int h = 0; h <= QM; ++h)
        if (h <= q) acc = fma4(Nv[h], row[h], acc);
    return acc;
}

// Column set-up shared by forward and backward: this lane's v-span and
// basis, and the tile's control-column range [j0, j0 + ncols).
template <int QM>
__device__ __forceinline__ int tile_columns(const Surf& s, int q, int col0, float Nv[QM + 1], bool& act,
                                            int& j0, int& ncols) {
    const int lane = lane_id();
    const int b = col0 + lane;
    act = b < s.nv_s;
    const int kb = sample_basis_rt<QM>(s.kv, s.nv_c, s.vs[act ? b : s.nv_s - 1], q, Nv);
    const int nact = min(kWave, s.nv_s - col0);
    const int kfirst = bcast_lane(kb, 0);
    const int klast = bcast_lane(kb, nact - 1);
    j0 = kfirst - q;
    ncols = klast - j0 + 1;
    return kb;
}

// Copy a knot vector (<= kWG entries) into this wave's LDS, so that span
// searches and basis evaluations read LDS instead of chasing global loads.
__device__ __forceinline__ const float* stage_knots(const float* __restrict__ U, int n, float* dst) {
    const int lane = lane_id();
    float v[kWG / kWave];
#pragma unroll
    for (int m = 0; m < kWG / kWave; ++m) {
        const int i = lane + m * kWave;
        if (i < n) v[m] = U[i];
    }
#pragma unroll
    for (int m = 0; m < kWG / kWave; ++m) {
        const int i = lane + m * kWave;
        if (i < n) dst[i] = v[m];
    }
    return dst;
}

// The first P+2 ring rows (window rows k-P .. k and the next one), loads
// issued together so the tile waits for one memory latency, not P+2.
template <int P>
__device__ __forceinline__ void stage_ring(const Surf& s, const Ring& rg, int k) {
    const int lane = lane_id();
    float4 v[P + 2];
#pragma unroll
    for (int r = 0; r < P + 2; ++r) {
        const int i = k - P + r;
        if (i < s.nu_c && lane < rg.ncols) v[r] = load_pw(s, i, rg.j0 + lane);
    }
#pragma unroll
    for (int r = 0; r < P + 2; ++r)
        if (lane < rg.ncols) ring_row(rg, k - P + r)[lane] = v[r];
}

__device__ __forceinline__ Ring make_ring(float4* base, int j0, int ncols, int p) {
    Ring rg;
    rg.base = base;
    rg.j0 = j0;
    rg.ncols = ncols;
    rg.nslots = p + 2;
    rg.on = ncols <= kWave && (p + 2) * ncols <= kRingCap;
    return rg;
}

// --------------------------------------------------------------------------
// forward tile
// --------------------------------------------------------------------------
// per-wave LDS of the forward tile
struct FwdLds {
    float4 ring[kRingCap];
    float knots[2][kWG];
};

template <int P, int QM>
__device__ __forceinline__ void fwd_tile(const Surf& sg, int q, int col0, int row0, int row1,
                                         float* __restrict__ pts, FwdLds* lds) {
    const int lane = lane_id();
    const int b = col0 + lane;
    // knots from LDS from here on
    Surf s = sg;
    s.ku = stage_knots(sg.ku, sg.nu_c + P + 1, lds->knots[0]);
    s.kv = stage_knots(sg.kv, sg.nv_c + q + 1, lds->knots[1]);
    wave_lds_sync();
    float4* ring_lds = lds->ring;
    float Nv[QM + 1];
    bool act;
    int j0, ncols;
    const int kb = tile_columns<QM>(s, q, col0, Nv, act, j0, ncols);
    const int jb = kb - q;
    const Ring rg = make_ring(ring_lds, j0, ncols, P);

    float4 R[P + 1];
    RowPrefetch pf;
    int cur = -1;  // window rows cur-P .. cur; ring holds rows up to nxt-1
    int nxt = 0;
    float u_next = s.us[min(row0 + lane, row1 - 1)];
    for (int a0 = row0; a0 < row1; a0 += kWave) {
        const int nr = min(kWave, row1 - a0);
        float Nu_l[P + 1];
        const int ka_l = sample_basis<P>(s.ku, s.nu_c, u_next, Nu_l);
        if (a0 + kWave < row1) u_next = s.us[min(a0 + kWave + lane, row1 - 1)];
        for (int t = 0; t < nr; ++t) {
            const int ka = bcast_lane(ka_l, t);
            if (cur < 0) {
                // first row: stage rows ka-P .. ka+1, prefetch ka+2
                if (rg.on) {
                    stage_ring<P>(s, rg, ka);
                    wave_lds_sync();
                    nxt = ka + 2;
                    prefetch_row(s, rg, nxt, pf);
                }
                cur = ka;
#pragma unroll
                for (int r = 0; r <= P; ++r) R[r] = ring_contract<QM>(s, rg, ka - P + r, jb, Nv, q);
            } else {
                while (cur < ka) {
#pragma unroll
                    for (int r = 0; r < P; ++r) R[r] = R[r + 1];
                    ++cur;
                    R[P] = ring_contract<QM>(s, rg, cur, jb, Nv, q);
                    if (rg.on) {
                        wave_lds_sync();
                        store_row(rg, nxt, pf);  // replaces row cur-P-1, now outside the window
                        wave_lds_sync();
                        ++nxt;
                        prefetch_row(s, rg, nxt, pf);
                    }
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

// per-wave LDS of the backward tile, sized for degrees p <= PM, q <= QM
template <int PM, int QM>
struct BwdLdsT {
    float knots[2][kWG];
    float4 ring[kRingCap];
    float4 col[kWave * (QM + 1)];           // segment sums, [head lane][h]
    short head_of[kWG];                     // key offset -> head lane, or -1
    float ebuf[kEBatch * 4 * (PM + 1)];     // 16-lane partials of dL/dNu
};

// pointers into one wave's BwdLdsT
struct BwdLds {
    float* knots[2];
    float4* ring;
    float4* col;
    short* head_of;
    float* ebuf;
};

template <int PM, int QM>
__device__ __forceinline__ BwdLds bwd_lds(BwdLdsT<PM, QM>* t) {
    BwdLds l;
    l.knots[0] = t->knots[0];
    l.knots[1] = t->knots[1];
    l.ring = t->ring;
    l.col = t->col;
    l.head_of = t->head_of;
    l.ebuf = t->ebuf;
    return l;
}

// Flush control row i (accumulator G) of the tile: dV partial and the rect
// row i - i0 of dL/dPw.
template <int QM>
__device__ __forceinline__ void flush_row(const Surf& s, BwdState<QM>& st, const Ring& rg, int i, int i0,
                                          float4 G, float4* __restrict__ rect, BwdLds* L, bool want_pw,
                                          bool want_kv) {
    const int lane = lane_id();
    const int q = st.q;
    if (want_kv) {
        if (rg.on) {
            const float4* row = ring_row(rg, i) + (st.jb - rg.j0);
#pragma unroll
            for (int h = 0; h <= QM; ++h)
                if (h <= q) st.f[h] += dot4(row[h], G);
        } else {
#pragma unroll
            for (int h = 0; h <= QM; ++h)
                if (h <= q) st.f[h] += dot4(load_pw(s, i, st.jb + h), G);
        }
    }
    if (!want_pw) return;
    // segmented inclusive scan over lanes sharing a v-span, one h at a time
#pragma unroll
    for (int h = 0; h <= QM; ++h) {
        if (h > q) continue;
        const float c = st.act ? st.Nv[h] : 0.f;
        float4 x = make_float4(c * G.x, c * G.y, c * G.z, c * G.w);
        for (int step = 0, d = 1; step < st.nsteps; ++step, d <<= 1) {
            const bool take = (lane - d) >= st.seg_first;
            float4 y;
            y.x = __shfl_up(x.x, d, kWave);
            y.y = __shfl_up(x.y, d, kWave);
            y.z = __shfl_up(x.z, d, kWave);
            y.w = __shfl_up(x.w, d, kWave);
            if (take) {
                x.x += y.x;
                x.y += y.y;
                x.z += y.z;
                x.w += y.w;
            }
        }
        if (st.head) L->col[lane * (QM + 1) + h] = x;
    }
    wave_lds_sync();
    // control column j = j0 + c gathers keys kfirst + c - h
    for (int c = lane; c < st.ncols; c += kWave) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int h = 0; h <= QM; ++h) {
            const int o = c - h;
            const int hl = (h <= q && o >= 0 && o < st.nkeys) ? (int)L->head_of[o] : -1;
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
    int j0, ncols;
    st.kb = tile_columns<QM>(s, q, col0, st.Nv, st.act, j0, ncols);
    st.jb = st.kb - q;
#pragma unroll
    for (int h = 0; h <= QM; ++h) st.f[h] = 0.f;
    const int kfirst = j0 + q;
    st.j0 = j0;
    st.ncols = ncols;
    st.nkeys = ncols - q;
    st.key_off = st.kb - kfirst;
    const int nact = min(kWave, s.nv_s - col0);
    const int kb_next = __shfl_down(st.kb, 1, kWave);
    st.head = st.act && (lane == nact - 1 || kb_next != st.kb);
    {   // first lane of the segment: the largest segment start at or below this lane
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
    for (int o = lane; o < st.nkeys; o += kWave) L->head_of[o] = (short)-1;
    wave_lds_sync();
    if (st.head) L->head_of[st.key_off] = (short)lane;
    wave_lds_sync();
}

// Finish a batch of nb rows of dL/dNu: add the four 16-lane partials of
// each (row, r) in a fixed order and store them contiguously.
template <int P>
__device__ __forceinline__ void flush_e(BwdLds* L, int nb, float* __restrict__ e_out) {
    const int lane = lane_id();
    wave_lds_sync();
    for (int idx = lane; idx < nb * (P + 1); idx += kWave) {
        const int t = idx / (P + 1), r = idx - t * (P + 1);
        const float* e = L->ebuf + (t * 4) * (P + 1) + r;
        e_out[idx] = ((e[0] + e[P + 1]) + e[2 * (P + 1)]) + e[3 * (P + 1)];
    }
    wave_lds_sync();
}

template <int P, int QM>
__device__ __forceinline__ void bwd_rows(const Surf& s, BwdState<QM>& st, int col0, int row0, int row1,
                                         const float* __restrict__ gpts, SlotView out, BwdLds* L,
                                         unsigned mask) {
    constexpr int D = 4;  // rows of dL/dS in flight
    const int lane = lane_id();
    const bool want_pw = (mask & 3u) != 0;
    const bool want_ku = (mask & 4u) != 0;
    const bool want_kv = (mask & 8u) != 0;
    const int q = st.q;
    const int b = col0 + lane;
    const Ring rg = make_ring(L->ring, st.j0, st.ncols, P);
    float4 R[P + 1], G[P + 1];
    RowPrefetch pf;
    int cur = -1, i0 = 0, nxt = 0;
    // Slide the window until its last row is `target`, flushing every row
    // that leaves it.  Rows past the last control row are never loaded; the
    // end-of-tile drain uses this with target = cur + P + 1.
    auto advance = [&](int target) {
        while (cur < target) {
            flush_row<QM>(s, st, rg, cur - P, i0, G[0], out.rect, L, want_pw, want_kv);
#pragma unroll
            for (int r = 0; r < P; ++r) {
                R[r] = R[r + 1];
                G[r] = G[r + 1];
            }
            ++cur;
            G[P] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (cur < s.nu_c) R[P] = ring_contract<QM>(s, rg, cur, st.jb, st.Nv, q);
            if (rg.on && nxt < s.nu_c) {
                wave_lds_sync();
                store_row(rg, nxt, pf);  // replaces the row just flushed
                wave_lds_sync();
                ++nxt;
                prefetch_row(s, rg, nxt, pf);
            }
        }
    };
    // dL/dS of the next D rows, in flight while the current rows are processed
    float3 gq[D];
    auto load_g = [&](int a) {
        float3 v = make_float3(0.f, 0.f, 0.f);
        if (st.act && a < row1) {
            const float* gp = gpts + 3 * ((size_t)a * s.nv_s + b);
            v = make_float3(gp[0], gp[1], gp[2]);
        }
        return v;
    };
#pragma unroll
    for (int j = 0; j < D; ++j) gq[j] = load_g(row0 + j);
    float u_next = s.us[min(row0 + lane, row1 - 1)];
    for (int a0 = row0; a0 < row1; a0 += kWave) {
        const int nr = min(kWave, row1 - a0);
        float Nu_l[P + 1];
        const int ka_l = sample_basis<P>(s.ku, s.nu_c, u_next, Nu_l);
        if (a0 + kWave < row1) u_next = s.us[min(a0 + kWave + lane, row1 - 1)];
        int eb = 0;  // rows in the current dL/dNu batch
        for (int t0 = 0; t0 < nr; t0 += D) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int t = t0 + j;
                if (t >= nr) break;
                const int ka = bcast_lane(ka_l, t);
                if (cur < 0) {
                    cur = ka;
                    i0 = ka - P;
                    if (rg.on) {
                        stage_ring<P>(s, rg, ka);
                        wave_lds_sync();
                        nxt = ka + 2;
                        prefetch_row(s, rg, nxt, pf);
                    }
#pragma unroll
                    for (int r = 0; r <= P; ++r) {
                        R[r] = ring_contract<QM>(s, rg, ka - P + r, st.jb, st.Nv, q);
                        G[r] = make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                } else {
                    // rows are non-decreasing, so the window only moves forward
                    advance(ka);
                }
                const float3 g = gq[j];
                gq[j] = load_g(a0 + t + D);
                float Nu[P + 1];
#pragma unroll
                for (int r = 0; r <= P; ++r) Nu[r] = bcast_lane(Nu_l[r], t);
                // recompute S' (nothing is saved by the forward)
                float4 sp = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int r = 0; r <= P; ++r) sp = fma4(Nu[r], R[r], sp);
                const float rw = recip(sp.w);
                const float cx = g.x * rw, cy = g.y * rw, cz = g.z * rw;
                const float cw = -(cx * sp.x + cy * sp.y + cz * sp.z) * rw;
                const float4 hv = make_float4(cx, cy, cz, cw);
#pragma unroll
                for (int r = 0; r <= P; ++r) G[r] = fma4(Nu[r], hv, G[r]);
                if (want_ku) {
#pragma unroll
                    for (int r = 0; r <= P; ++r) {
                        const float e = row16_sum(dot4(R[r], hv));
                        if ((lane & 15) == 0) L->ebuf[(eb * 4 + (lane >> 4)) * (P + 1) + r] = e;
                    }
                    if (++eb == kEBatch) {
                        flush_e<P>(L, eb, out.e + (size_t)(a0 + t + 1 - eb - row0) * (P + 1));
                        eb = 0;
                    }
                }
            }
        }
        if (want_ku && eb > 0) flush_e<P>(L, eb, out.e + (size_t)(a0 + nr - eb - row0) * (P + 1));
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

// Knots of the tile's surface into LDS; returns the surface view that reads them.
__device__ __forceinline__ Surf bwd_stage_knots(const Surf& sg, int p, int q, BwdLds* L) {
    Surf s = sg;
    s.ku = stage_knots(sg.ku, sg.nu_c + p + 1, L->knots[0]);
    s.kv = stage_knots(sg.kv, sg.nv_c + q + 1, L->knots[1]);
    wave_lds_sync();
    return s;
}

template <int P, int QM>
__device__ __forceinline__ void bwd_tile(const Surf& sg, int q, int col0, int row0, int row1,
                                         const float* __restrict__ gpts, SlotView out, BwdLds* L, unsigned mask) {
    const Surf s = bwd_stage_knots(sg, P, q, L);
    BwdState<QM> st;
    bwd_columns<QM>(s, q, col0, st, L);
    bwd_rows<P, QM>(s, st, col0, row0, row1, gpts, out, L, mask);
}

// --------------------------------------------------------------------------
// finalize: one workgroup (kWG threads) per surface
// --------------------------------------------------------------------------
constexpr int kFinMaxTiles = 256;  // tile headers staged in LDS (more: read from global)
constexpr int kFinCp = 8;          // control points per thread per pass

struct FinLds {
    float knots[kWG];
    int4 hdr[kFinMaxTiles];
    float contrib[kWG * (2 * kMaxDeg + 2)];  // per sample, knot-window adjoints
    int span[kWG];
};

// Tiles of one surface in natural order (row blocks outer, 64-column blocks
// inner): slot pointer, column start and row range of tile t.
struct TileRef {
    const char* slot;
    int col0, row0, row1;
    int alloc_rows;  // rows the slot was sized for (>= row1 - row0)
};

// Knot gradient of one direction: for every sample x_a of the direction,
// coef(a)[r] = dL/dN_{k_a-D+r}(x_a) is turned into per-knot adjoints by
// basis_knot_adjoint (FP64); the adjoints are then summed over samples in
// sample order (chunks of kWG samples staged in LDS), one thread per knot.
template <int D, class CoefAt>
__device__ __forceinline__ void knot_gradient(const float* __restrict__ Ug, int nc, const float* __restrict__ xs,
                                              int ns, CoefAt coef_at, float* __restrict__ gout, FinLds* L) {
    constexpr int W = 2 * D + 2;
    const int tid = threadIdx.x;
    const int nk = nc + D + 1;
    const int n = nc - 1;
    __syncthreads();
    if (tid < nk) L->knots[tid] = Ug[tid];
    __syncthreads();
    const float* U = L->knots;
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
            for (int t = 0; t < W; ++t) L->contrib[tid * W + t] = (float)g[t];
        }
        L->span[tid] = k;
        __syncthreads();
        const int cnt = min(kWG, ns - a0);
        if (tid < nk) {
            for (int r = 0; r < cnt; ++r) {
                const int t = tid - (L->span[r] - D);
                if (t >= 0 && t < W) acc += (double)L->contrib[r * W + t];
            }
        }
        __syncthreads();
    }
    if (tid < nk) gout[tid] = (float)acc;
}

template <int P, int Q, class TileAt>
__device__ __forceinline__ void finalize_surface(const Surf& s, int ntiles, TileAt tile_at, float* __restrict__ gctrl,
                                                 float* __restrict__ gw, float* __restrict__ gku,
                                                 float* __restrict__ gkv, unsigned mask, FinLds* L) {
    const int tid = threadIdx.x;
    const size_t rect_bytes = 16 * (size_t)s.nu_c * s.nv_c;
    const int ncb = (s.nv_s + kWave - 1) / kWave;
    const int rows = ntiles > 0 ? tile_at(0).alloc_rows : 1;
    const int nrb = ncb > 0 ? ntiles / ncb : 0;
    const bool hdr_lds = ntiles <= kFinMaxTiles;
    if (hdr_lds)
        for (int t = tid; t < ntiles; t += kWG) L->hdr[t] = *reinterpret_cast<const int4*>(tile_at(t).slot);
    __syncthreads();
    // dL/dP and dL/dw from the tile rectangles, tiles in fixed order
    if (mask & 3u) {
        const int ncp = s.nu_c * s.nv_c;
        for (int base = 0; base < ncp; base += kWG * kFinCp) {
            float4 acc[kFinCp];
            int ii[kFinCp], jj[kFinCp];
#pragma unroll
            for (int c = 0; c < kFinCp; ++c) {
                acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
                const int ij = base + c * kWG + tid;
                ii[c] = ij / s.nv_c;
                jj[c] = ij - ii[c] * s.nv_c;
            }
            for (int t = 0; t < ntiles; ++t) {
                const char* slot = tile_at(t).slot;
                const int4 h = hdr_lds ? L->hdr[t] : *reinterpret_cast<const int4*>(slot);
                const float4* rect = reinterpret_cast<const float4*>(slot + 16);
                const int pitch = h.w - h.z + 1;
#pragma unroll
                for (int c = 0; c < kFinCp; ++c) {
                    const int ij = base + c * kWG + tid;
                    if (ij < ncp && ii[c] >= h.x && ii[c] <= h.y && jj[c] >= h.z && jj[c] <= h.w) {
                        const float4 v = rect[(size_t)(ii[c] - h.x) * pitch + (jj[c] - h.z)];
                        acc[c].x += v.x;
                        acc[c].y += v.y;
                        acc[c].z += v.z;
                        acc[c].w += v.w;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < kFinCp; ++c) {
                const int ij = base + c * kWG + tid;
                if (ij >= ncp) continue;
                const float wt = s.w[ij];
                const float* pc = s.ctrl + 3 * ij;
                if (mask & 1u) {
                    gctrl[3 * ij + 0] = wt * acc[c].x;
                    gctrl[3 * ij + 1] = wt * acc[c].y;
                    gctrl[3 * ij + 2] = wt * acc[c].z;
                }
                if (mask & 2u) gw[ij] = pc[0] * acc[c].x + pc[1] * acc[c].y + pc[2] * acc[c].z + acc[c].w;
            }
        }
    }
    // dL/dU: e(a) = sum over the column blocks of a's row block
    if (mask & 4u) {
        auto coef = [&](int a, double e[P + 1]) {
#pragma unroll
            for (int r = 0; r <= P; ++r) e[r] = 0.0;
            const int rb = a / rows;
            for (int cb = 0; cb < ncb; ++cb) {
                const TileRef tr = tile_at(rb * ncb + cb);
                const float* ev = reinterpret_cast<const float*>(tr.slot + 16 + rect_bytes) +
                                  (size_t)(a - tr.row0) * (P + 1);
#pragma unroll
                for (int r = 0; r <= P; ++r) e[r] += (double)ev[r];
            }
        };
        knot_gradient<P>(s.ku, s.nu_c, s.us, s.nu_s, coef, gku, L);
    }
    // dL/dV: f(b) = sum over the row blocks of b's column block
    if (mask & 8u) {
        auto coef = [&](int b, double f[Q + 1]) {
#pragma unroll
            for (int h = 0; h <= Q; ++h) f[h] = 0.0;
            const int cb = b / kWave;
            for (int rb = 0; rb < nrb; ++rb) {
                const TileRef tr = tile_at(rb * ncb + cb);
                const float* fv = reinterpret_cast<const float*>(
                    tr.slot + 16 + rect_bytes + align16(sizeof(float) * (size_t)tr.alloc_rows * (P + 1)));
#pragma unroll
                for (int h = 0; h <= Q; ++h) f[h] += (double)fv[(b - tr.col0) * (Q + 1) + h];
            }
        };
        knot_gradient<Q>(s.kv, s.nv_c, s.vs, s.nv_s, coef, gkv, L);
    }
}

}  // namespace nd
