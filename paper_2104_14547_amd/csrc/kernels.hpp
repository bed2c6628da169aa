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
// the tile and is *flushed*: f_h(b) += Pw[i][kb-q+h] . G_i(b) builds
// dL/dNv_h(b), and G_i(b) itself is stored, one float4 per lane, in the
// tile's workspace slot, beside a table of the tile's column spans and basis.
//
// Gather, a kernel of its own: the stored G_i are contracted along v,
// dL/dPw[i][j] = sum_b Nv_j(v_b) G_i(b), into the tile's partial dL/dPw
// rectangle, a small banded matrix product (control columns x 64 samples,
// times 64 samples x 4 values per control row) done on the matrix cores.
// It is kept out of the row loop, whose registers are all in use.  No
// atomics: each value is
// written once to a tile-indexed workspace slot, and the finalize pass adds
// slots in a fixed order, so results are bitwise reproducible and do not
// depend on which wave ran which tile.
//
// Finalize, one wave per surface: dL/dPw = sum of tile rectangles;
// dL/dP = w dL/dPw_xyz, dL/dw = P . dL/dPw_xyz + dL/dPw_w; dL/dU_k by the
// reverse-mode knot derivative of each row's basis weighted with e(a)
// (Sec. 3.2.1), dL/dV_k likewise with f(b).
#pragma once
#include <type_traits>

#include "device.hpp"
#include "launch.hpp"

namespace nd {

// --------------------------------------------------------------------------
// workspace layout of one backward tile (bytes from the slot start):
//   [0, 16)                      int4 header {i0, i1, j0, j1}
//   [16, 32)                     float4 {cx, cy, cz, 0}: the tile's frame origin
//   [32, 32 + 16*nu_c*nv_c)      float4 rect [(i1-i0+1)][(j1-j0+1)]
//   then float e[rows][P+1], then float f[64][Q+1] (each 16-byte aligned),
//   then the column table: int first[64] (first control column, tile-relative,
//   that sample column b touches; kGatherOff for inactive columns) and float
//   nv[64][Q+1] (its basis values Nv_h(v_b)),
//   then float4 gacc[nu_c][64]: the flushed accumulators G_i(b) of rows
//   i0..i1 (zero for inactive columns), which the gather contracts along v
//   into the rect.
// The rect holds dL/dPw in the tile's translated frame (control points
// P - c): the xyz part does not depend on the frame, the w part is
// dL/dw - (P - c) . dL/dPw_xyz of the tile's points.
// --------------------------------------------------------------------------
constexpr int kSlotHead = 32;
constexpr int kGatherOff = -(1 << 20);  // column-table entry of an inactive sample column

struct SlotView {
    int* hdr;
    float4* center;
    float4* rect;
    float* e;
    float* f;
    float4* gacc;
    int* ctab;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// byte offsets of the column table and of gacc in a slot
__host__ __device__ inline size_t slot_ctab_off(int p, int q, int nu_c, int nv_c, int rows) {
    size_t b = kSlotHead + 16 * (size_t)nu_c * nv_c;
    b += align16(sizeof(float) * (size_t)rows * (p + 1));
    b += align16(sizeof(float) * (size_t)kWave * (q + 1));
    return b;
}
__host__ __device__ inline size_t slot_gacc_off(int p, int q, int nu_c, int nv_c, int rows) {
    return slot_ctab_off(p, q, nu_c, nv_c, rows) + align16(sizeof(float) * (size_t)kWave * (q + 2));
}

__host__ __device__ inline size_t slot_bytes(int p, int q, int nu_c, int nv_c, int rows) {
    return slot_gacc_off(p, q, nu_c, nv_c, rows) + 16 * (size_t)nu_c * kWave;
}

__device__ __forceinline__ SlotView slot_view(char* base, int p, int q, int nu_c, int nv_c, int rows) {
    SlotView v;
    v.hdr = reinterpret_cast<int*>(base);
    v.center = reinterpret_cast<float4*>(base + 16);
    v.rect = reinterpret_cast<float4*>(base + kSlotHead);
    char* e = base + kSlotHead + 16 * (size_t)nu_c * nv_c;
    v.e = reinterpret_cast<float*>(e);
    v.f = reinterpret_cast<float*>(e + align16(sizeof(float) * (size_t)rows * (p + 1)));
    v.gacc = reinterpret_cast<float4*>(base + slot_gacc_off(p, q, nu_c, nv_c, rows));
    v.ctab = reinterpret_cast<int*>(base + slot_ctab_off(p, q, nu_c, nv_c, rows));
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
// control-row block: consecutive control rows of the tile's control columns
// j0 .. j0+ncols-1, as homogeneous points in LDS.  A block is loaded with all
// its loads in flight at once (one memory latency) and replaced only when
// the u-window leaves it, so the row loops below carry no pending loads.
// --------------------------------------------------------------------------
constexpr int kBlkCap = 320;                 // float4 entries per wave (5 KiB)
constexpr int kBlkPerLane = kBlkCap / kWave;  // entries each lane loads
constexpr int kEBatch = 8;                    // rows per batched reduction of dL/dN(u)

struct Block {
    float4* base;  // LDS, [rows][ncols]
    int j0, ncols;
    int lo, hi;    // staged control rows [lo, hi]
    int cap_rows;  // rows that fit
    bool on;       // false: the column range is too wide, read control points from global
};

__device__ __forceinline__ Block make_block(float4* base, int j0, int ncols, int p) {
    Block bk;
    bk.base = base;
    bk.j0 = j0;
    bk.ncols = ncols;
    bk.lo = 0;
    bk.hi = -1;
    bk.cap_rows = kBlkCap / max(ncols, 1);
    bk.on = bk.cap_rows >= p + 1;
    return bk;
}

// Load control rows [lo, min(lo + cap_rows, nu_c) - 1] into the block.
__device__ __forceinline__ void stage_block(const Surf& s, Block& bk, int lo) {
    const int lane = lane_opaque();
    bk.lo = lo;
    bk.hi = min(lo + bk.cap_rows, s.nu_c) - 1;
    const int n = (bk.hi - bk.lo + 1) * bk.ncols;
    constexpr int kRound = kBlkPerLane / 2;  // loads in flight per lane per round
#pragma unroll
    for (int m0 = 0; m0 < kBlkPerLane; m0 += kRound) {
        if (m0 * kWave >= n) break;
        float4 raw[kRound];
#pragma unroll
        for (int m = 0; m < kRound; ++m) {
            const int e = lane + (m0 + m) * kWave;
            if (e < n) {
                const int r = small_div(e, bk.ncols), c = e - r * bk.ncols;
                const int ij = (lo + r) * s.nv_c + bk.j0 + c;
                const float* cp = s.ctrl + 3 * ij;
                raw[m] = make_float4(cp[0], cp[1], cp[2], s.w[ij]);
            }
        }
#pragma unroll
        for (int m = 0; m < kRound; ++m) {
            const int e = lane + (m0 + m) * kWave;
            if (e < n)
                bk.base[e] = make_float4(raw[m].x * raw[m].w, raw[m].y * raw[m].w, raw[m].z * raw[m].w, raw[m].w);
        }
    }
    wait_vmem();
    wave_lds_sync();
}

// Make sure rows [need_lo, need_hi] are staged (need_hi - need_lo < cap_rows).
// The row loops are compiled twice, with BLK = bk.on known: the block
// version has no global loads between restagings, so no wait on memory
// (which on gfx9 also waits for this wave's earlier stores) sits in it.
template <bool BLK>
__device__ __forceinline__ void ensure_rows(const Surf& s, Block& bk, int need_lo, int need_hi) {
    if constexpr (BLK) {
        if (need_lo < bk.lo || need_hi > bk.hi) {
            wave_lds_sync();
            stage_block(s, bk, need_lo);
        }
    }
}

// Homogeneous control points of row i starting at this lane's first column
// jb: a pointer into the block.
__device__ __forceinline__ const float4* block_row(const Block& bk, int i, int jb) {
    return bk.base + (i - bk.lo) * bk.ncols + (jb - bk.j0);
}

// R_i(b) for this lane's column from the block (or from global memory).
template <int QM, bool BLK>
__device__ __forceinline__ float4 blk_contract(const Surf& s, const Block& bk, int i, int jb,
                                               const float Nv[QM + 1], int q) {
    if constexpr (!BLK) return row_contract<QM>(s, i, jb, Nv, q);
    const float4* row = block_row(bk, i, jb);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int h = 0; h <= QM; ++h)
        if (h <= q) acc = fma4(Nv[h], row[h], acc);
    return acc;
}

// First inputs of a tile, fetched together (one memory latency): both knot
// vectors (<= kWG entries each) into this wave's LDS, so that span searches
// and basis evaluations read LDS; the lane's v parameter; and the u
// parameter of the lane's row in the tile's first 64-row chunk.
struct TileIn {
    float v;   // vs[col0 + lane] (clamped to the last column)
    float u0;  // us[row0 + lane] (clamped to the chunk)
};

__device__ __forceinline__ TileIn stage_tile(const Surf& sg, int p, int q, int col0, int row0, int row1,
                                             float* ku_dst, float* kv_dst) {
    const int lane = lane_id();
    const int nU = sg.nu_c + p + 1, nV = sg.nv_c + q + 1;
    float a[kWG / kWave], c[kWG / kWave];
#pragma unroll
    for (int m = 0; m < kWG / kWave; ++m) {
        const int i = lane + m * kWave;
        if (i < nU) a[m] = sg.ku[i];
        if (i < nV) c[m] = sg.kv[i];
    }
    TileIn in;
    in.v = sg.vs[min(col0 + lane, sg.nv_s - 1)];
    in.u0 = sg.us[row0 + min(lane, min(kWave, row1 - row0) - 1)];
#pragma unroll
    for (int m = 0; m < kWG / kWave; ++m) {
        const int i = lane + m * kWave;
        if (i < nU) ku_dst[i] = a[m];
        if (i < nV) kv_dst[i] = c[m];
    }
    wait_vmem();
    wave_lds_sync();
    return in;
}

// Fixed-knot tables: the column's span and basis, and those of the lane's
// row in the tile's first 64-row chunk, loaded before stage_tile so that
// its final wait covers them (one memory latency for all first inputs).
template <int QM>
struct ColPre {
    int k;
    float N[QM + 1];
};
template <int P>
struct RowPre {
    int k;
    float N[P + 1];
};
template <int QM>
__device__ __forceinline__ void col_prefetch(const Surf& s, int q, int col0, ColPre<QM>& c) {
    const int bc = min(col0 + lane_id(), s.nv_s - 1);
    c.k = s.tsv[bc];
#pragma unroll
    for (int h = 0; h <= QM; ++h) c.N[h] = h <= q ? s.tbv[(size_t)bc * (q + 1) + h] : 0.f;
}
template <int P>
__device__ __forceinline__ void row_prefetch(const Surf& s, int row0, int row1, RowPre<P>& r) {
    const int ra = row0 + min(lane_id(), min(kWave, row1 - row0) - 1);
    r.k = s.tsu[ra];
#pragma unroll
    for (int i = 0; i <= P; ++i) r.N[i] = s.tbu[(size_t)ra * (P + 1) + i];
}

// Column set-up shared by forward and backward: this lane's v-span and
// basis, and the tile's control-column range [j0, j0 + ncols).
template <int QM, bool TAB = false>
__device__ __forceinline__ int tile_columns(const Surf& s, int q, int col0, float vb, float Nv[QM + 1], bool& act,
                                            int& j0, int& ncols, const ColPre<QM>* pre = nullptr) {
    const int lane = lane_id();
    const int b = col0 + lane;
    act = b < s.nv_s;
    int kb;
    if constexpr (TAB) {  // fixed knots: the column's span and basis, prefetched from the table
        kb = pre->k;
#pragma unroll
        for (int h = 0; h <= QM; ++h) Nv[h] = pre->N[h];
    } else {
        kb = sample_basis_rt<QM>(s.kv, s.nv_c, vb, q, Nv);
    }
    const int nact = min(kWave, s.nv_s - col0);
    const int kfirst = bcast_lane(kb, 0);
    const int klast = bcast_lane(kb, nact - 1);
    j0 = kfirst - q;
    ncols = klast - j0 + 1;
    return kb;
}

// --------------------------------------------------------------------------
// forward tile
// --------------------------------------------------------------------------
struct FwdLds {
    float4 blk[kBlkCap];
    float knots[2][kWG];
};

// The span and basis of row a0 + min(lane, nr - 1): from the fixed-knot
// table, or evaluated from the parameter ua.
template <int P, bool TAB>
__device__ __forceinline__ int row_basis(const Surf& s, int a0, int nr, float ua, float Nu_l[P + 1],
                                         const RowPre<P>* pre) {
    if constexpr (TAB) {
        if (pre) {  // the tile's first chunk: prefetched with the tile's first inputs
#pragma unroll
            for (int r = 0; r <= P; ++r) Nu_l[r] = pre->N[r];
            return pre->k;
        }
        const int ra = a0 + min(lane_id(), nr - 1);
#pragma unroll
        for (int r = 0; r <= P; ++r) Nu_l[r] = s.tbu[(size_t)ra * (P + 1) + r];
        return s.tsu[ra];
    } else {
        return sample_basis<P>(s.ku, s.nu_c, ua, Nu_l);
    }
}

template <int P, int QM, bool BLK, bool TAB = false>
__device__ __forceinline__ void fwd_rows(const Surf& s, Block& bk, const float Nv[QM + 1], int q, int jb, bool act,
                                         int row0, int row1, float u0, float* __restrict__ orow, size_t ostride,
                                         const RowPre<P>* rpre = nullptr) {
    const int lane = lane_id();
    float4 R[P + 1];
    int cur = -1;  // window rows cur-P .. cur
    for (int a0 = row0; a0 < row1; a0 += kWave) {
        const int nr = min(kWave, row1 - a0);
        float Nu_l[P + 1];
        const float ua = TAB ? 0.f : (a0 == row0 ? u0 : s.us[a0 + min(lane, nr - 1)]);
        const int ka_l = row_basis<P, TAB>(s, a0, nr, ua, Nu_l, a0 == row0 ? rpre : nullptr);
        for (int t = 0; t < nr; ++t) {
            const int ka = bcast_lane(ka_l, t);
            if (ka != cur) {
                ensure_rows<BLK>(s, bk, ka - P, ka);
                if (cur >= 0 && ka > cur && ka - cur <= P) {
                    do {
#pragma unroll
                        for (int r = 0; r < P; ++r) R[r] = R[r + 1];
                        ++cur;
                        R[P] = blk_contract<QM, BLK>(s, bk, cur, jb, Nv, q);
                    } while (cur < ka);
                } else {
                    cur = ka;
#pragma unroll
                    for (int r = 0; r <= P; ++r) R[r] = blk_contract<QM, BLK>(s, bk, ka - P + r, jb, Nv, q);
                }
            }
            if (t + 1 < nr && bcast_lane(ka_l, t + 1) == ka) {
                // two rows on the same window: their independent chains overlap
                float4 acc = make_float4(0.f, 0.f, 0.f, 0.f), acc2 = acc;
#pragma unroll
                for (int r = 0; r <= P; ++r) {
                    acc = fma4(bcast_lane(Nu_l[r], t), R[r], acc);
                    acc2 = fma4(bcast_lane(Nu_l[r], t + 1), R[r], acc2);
                }
                const float rw = recip_fast(acc.w), rw2 = recip_fast(acc2.w);
                if (act) {
                    store3(orow, acc.x * rw, acc.y * rw, acc.z * rw);
                    store3(orow + ostride, acc2.x * rw2, acc2.y * rw2, acc2.z * rw2);
                }
                orow += 2 * ostride;
                ++t;
                continue;
            }
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int r = 0; r <= P; ++r) acc = fma4(bcast_lane(Nu_l[r], t), R[r], acc);
            const float rw = recip_fast(acc.w);
            if (act) store3(orow, acc.x * rw, acc.y * rw, acc.z * rw);
            orow += ostride;
        }
    }
}

template <int P, int QM, bool TAB = false>
__device__ __forceinline__ void fwd_tile(const Surf& sg, int q, int col0, int row0, int row1,
                                         float* __restrict__ pts, FwdLds* lds) {
    const int lane = lane_id();
    const int b = col0 + lane;
    // knots from LDS from here on
    Surf s = sg;
    ColPre<QM> cpre;
    RowPre<P> rpre;
    if constexpr (TAB) {
        col_prefetch<QM>(sg, q, col0, cpre);
        row_prefetch<P>(sg, row0, row1, rpre);
    }
    const TileIn in = stage_tile(sg, P, q, col0, row0, row1, lds->knots[0], lds->knots[1]);
    s.ku = lds->knots[0];
    s.kv = lds->knots[1];
    float Nv[QM + 1];
    bool act;
    int j0, ncols;
    const int kb = tile_columns<QM, TAB>(s, q, col0, in.v, Nv, act, j0, ncols, &cpre);
    const int jb = kb - q;
    Block bk = make_block(lds->blk, j0, ncols, P);
    float* orow = pts + 3 * ((size_t)row0 * s.nv_s + b);
    const size_t ostride = 3 * (size_t)s.nv_s;
    if (bk.on)
        fwd_rows<P, QM, true, TAB>(s, bk, Nv, q, jb, act, row0, row1, in.u0, orow, ostride, &rpre);
    else
        fwd_rows<P, QM, false, TAB>(s, bk, Nv, q, jb, act, row0, row1, in.u0, orow, ostride, &rpre);
}

// --------------------------------------------------------------------------
// parametric derivatives and unit normals (Appendix A, eq.
// NURBSuDerivative1: S_u = (A_u - S w_u) / w with A = sum N_i N_j Pw_ij the
// homogeneous point; the normals S_u x S_v / |S_u x S_v| are what surface
// offsetting moves points along, Sec. 4.3).  Same tiles as the forward, with
// two contracted windows per lane: R_i(b) with Nv and Rv_i(b) with dNv/dv.
// --------------------------------------------------------------------------
struct DerOut {
    float* pts;  // S      [nu_s][nv_s][3], or NULL
    float* du;   // dS/du  [nu_s][nv_s][3], or NULL
    float* dv;   // dS/dv  [nu_s][nv_s][3], or NULL
    float* nrm;  // unit normal (0 where S_u x S_v vanishes), or NULL
};

template <int P, int QM, bool BLK>
__device__ __forceinline__ void der_rows(const Surf& s, Block& bk, const float Nv[QM + 1], const float dNv[QM + 1],
                                         int q, int jb, bool act, int row0, int row1, float u0, const DerOut& o,
                                         size_t off, size_t ostride) {
    const int lane = lane_id();
    float4 R[P + 1], Rv[P + 1];
    int cur = -1;  // window rows cur-P .. cur
    for (int a0 = row0; a0 < row1; a0 += kWave) {
        const int nr = min(kWave, row1 - a0);
        float Nu_l[P + 1], dNu_l[P + 1];
        const float ua = a0 == row0 ? u0 : s.us[a0 + min(lane, nr - 1)];
        const int ka_l = sample_basis_d1<P>(s.ku, s.nu_c, ua, Nu_l, dNu_l);
        for (int t = 0; t < nr; ++t, off += ostride) {
            const int ka = bcast_lane(ka_l, t);
            if (ka != cur) {
                ensure_rows<BLK>(s, bk, ka - P, ka);
                if (cur >= 0 && ka > cur && ka - cur <= P) {
                    do {
#pragma unroll
                        for (int r = 0; r < P; ++r) {
                            R[r] = R[r + 1];
                            Rv[r] = Rv[r + 1];
                        }
                        ++cur;
                        R[P] = blk_contract<QM, BLK>(s, bk, cur, jb, Nv, q);
                        Rv[P] = blk_contract<QM, BLK>(s, bk, cur, jb, dNv, q);
                    } while (cur < ka);
                } else {
                    cur = ka;
#pragma unroll
                    for (int r = 0; r <= P; ++r) {
                        R[r] = blk_contract<QM, BLK>(s, bk, ka - P + r, jb, Nv, q);
                        Rv[r] = blk_contract<QM, BLK>(s, bk, ka - P + r, jb, dNv, q);
                    }
                }
            }
            float4 A = make_float4(0.f, 0.f, 0.f, 0.f), Au = A, Av = A;
#pragma unroll
            for (int r = 0; r <= P; ++r) {
                A = fma4(bcast_lane(Nu_l[r], t), R[r], A);
                Au = fma4(bcast_lane(dNu_l[r], t), R[r], Au);
                Av = fma4(bcast_lane(Nu_l[r], t), Rv[r], Av);
            }
            const float rw = recip(A.w);
            const float sx = A.x * rw, sy = A.y * rw, sz = A.z * rw;
            const float ux = (Au.x - sx * Au.w) * rw, uy = (Au.y - sy * Au.w) * rw, uz = (Au.z - sz * Au.w) * rw;
            const float vx = (Av.x - sx * Av.w) * rw, vy = (Av.y - sy * Av.w) * rw, vz = (Av.z - sz * Av.w) * rw;
            if (!act) continue;
            if (o.pts) store3(o.pts + off, sx, sy, sz);
            if (o.du) store3(o.du + off, ux, uy, uz);
            if (o.dv) store3(o.dv + off, vx, vy, vz);
            if (o.nrm) {
                const float nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
                const float l2 = nx * nx + ny * ny + nz * nz;
                const float il = l2 > 0.f ? __builtin_amdgcn_rsqf(l2) : 0.f;
                store3(o.nrm + off, nx * il, ny * il, nz * il);
            }
        }
    }
}

template <int P, int QM>
__device__ __forceinline__ void der_tile(const Surf& sg, int q, int col0, int row0, int row1, const DerOut& o,
                                         FwdLds* lds) {
    const int lane = lane_id();
    Surf s = sg;
    const TileIn in = stage_tile(sg, P, q, col0, row0, row1, lds->knots[0], lds->knots[1]);
    s.ku = lds->knots[0];
    s.kv = lds->knots[1];
    float Nv[QM + 1], dNv[QM + 1];
#pragma unroll
    for (int h = 0; h <= QM; ++h) Nv[h] = dNv[h] = 0.f;
    const int b = col0 + lane;
    const bool act = b < s.nv_s;
    int kb = 0;
    switch (q) {
#define ND_DV(D)                                                                        \
    case D:                                                                             \
        if constexpr (D <= QM) {                                                        \
            float n_[D + 1], d_[D + 1];                                                 \
            kb = sample_basis_d1<D>(s.kv, s.nv_c, in.v, n_, d_);                        \
            _Pragma("unroll") for (int h = 0; h <= D; ++h) { Nv[h] = n_[h]; dNv[h] = d_[h]; } \
        }                                                                               \
        break;
        ND_DV(1) ND_DV(2) ND_DV(3) ND_DV(4) ND_DV(5) ND_DV(6) ND_DV(7)
#undef ND_DV
        default: break;
    }
    const int nact = min(kWave, s.nv_s - col0);
    const int kfirst = bcast_lane(kb, 0), klast = bcast_lane(kb, nact - 1);
    const int j0 = kfirst - q;
    Block bk = make_block(lds->blk, j0, klast - j0 + 1, P);
    const size_t off = 3 * ((size_t)row0 * s.nv_s + b);
    const size_t ostride = 3 * (size_t)s.nv_s;
    if (bk.on)
        der_rows<P, QM, true>(s, bk, Nv, dNv, q, kb - q, act, row0, row1, in.u0, o, off, ostride);
    else
        der_rows<P, QM, false>(s, bk, Nv, dNv, q, kb - q, act, row0, row1, in.u0, o, off, ostride);
}

// --------------------------------------------------------------------------
// backward tile
// --------------------------------------------------------------------------
// per-lane state of a backward tile's row loop
template <int QM>
struct BwdState {
    float Nv[QM + 1];
    int kb, jb;
    bool act;
    int j0, ncols;    // rect column range
    int q;            // degree in v (uniform, <= QM)
    float f[QM + 1];  // dL/dNv_h(v_b) partial
    float cx, cy, cz; // the tile's frame origin (a control point of the tile, uniform)
};

// per-wave LDS of the backward tile's row loop, sized for degrees p <= PM
template <int PM, int QM>
struct BwdLdsT {
    float4 blk[kBlkCap];
    float knots[2][kWG];
    float ebuf[kEBatch * 4 * (PM + 1)];     // 16-lane partials of dL/dNu
};

// pointers into one wave's BwdLdsT
struct BwdLds {
    float4* blk;
    float* knots[2];
    float* ebuf;
};

template <int PM, int QM>
__device__ __forceinline__ BwdLds bwd_lds(BwdLdsT<PM, QM>* t) {
    BwdLds l;
    l.blk = t->blk;
    l.knots[0] = t->knots[0];
    l.knots[1] = t->knots[1];
    l.ebuf = t->ebuf;
    return l;
}

// Per-wave LDS of the gather: the current tile's column table, from which
// the lanes build their operands of the contraction.
template <int QM>
struct GatTab {
    int first[kWave];
    float nv[kWave * (QM + 1)];
};

// One step of a segmented inclusive scan on the four components:
// x += m * x[source lane], as one v_fmac_f32 per component that reads x
// through DPP (the compiler emits a separate v_mov_b32_dpp for this form).
// s_nop 1 gives the two wait states a DPP read needs after the last VALU
// write of its register; inside the block each component was written four
// instructions before it is read.
#define ND_SEG_STEP4(x, m, DPP)                                 \
    asm volatile("s_nop 1\n\t"                                 \
                 "v_fmac_f32_dpp %0, %0, %4 " DPP "\n\t"        \
                 "v_fmac_f32_dpp %1, %1, %4 " DPP "\n\t"        \
                 "v_fmac_f32_dpp %2, %2, %4 " DPP "\n\t"        \
                 "v_fmac_f32_dpp %3, %3, %4 " DPP                \
                 : "+v"(x.x), "+v"(x.y), "+v"(x.z), "+v"(x.w)    \
                 : "v"(m))

// Segmented inclusive scan over the wave (segments are runs of equal
// v-span): in-row Hillis-Steele steps (row_shr 1, 2, 4, 8), then the
// row_bcast 15 / 31 steps that carry runs across 16-lane rows.  After it,
// the last lane of each run holds the run's sum.  The step count and the
// cross-row flag are wave-uniform, so the steps are taken or skipped by
// scalar branches.  Lanes without a source lane (bound_ctrl) or in rows the
// step leaves out (row_mask) keep x.  Fixed order: deterministic.
template <class S>
__device__ __forceinline__ void seg_scan4(float4& x, const S& st) {
    if (st.nsteps > 0) ND_SEG_STEP4(x, st.m[0], "row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    if (st.nsteps > 1) ND_SEG_STEP4(x, st.m[1], "row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    if (st.nsteps > 2) ND_SEG_STEP4(x, st.m[2], "row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    if (st.nsteps > 3) ND_SEG_STEP4(x, st.m[3], "row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    if (st.cross) {
        ND_SEG_STEP4(x, st.m[4], "row_bcast:15 row_mask:0xa bank_mask:0xf");
        ND_SEG_STEP4(x, st.m[5], "row_bcast:31 row_mask:0xc bank_mask:0xf");
    }
}

// Runs of equal keys over the wave (keys non-decreasing with the lane): the
// multipliers of the DPP segmented scan, its wave-uniform step count and
// cross-row flag, and whether this lane is the last of its run.
struct Runs {
    float m[6];
    int nsteps;
    bool cross;
    bool head;
};

__device__ __forceinline__ Runs wave_runs(int key) {
    const int lane = lane_id();
    Runs r;
    const int next = __shfl_down(key, 1, kWave);
    const int prev = __shfl_up(key, 1, kWave);
    r.head = lane == kWave - 1 || next != key;
    const bool starts = lane == 0 || prev != key;
    // first lane of the run: the largest run start at or below this lane
    int f = starts ? lane : 0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(f, d, kWave);
        if (lane >= d) f = max(f, y);
    }
    // longest run inside one 16-lane row, and whether any run crosses rows
    const int row0 = lane & ~15;
    int len = lane - max(f, row0) + 1;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) len = max(len, __shfl_xor(len, d, kWave));
    int steps = 0;
    while ((1 << steps) < len) ++steps;
    r.nsteps = uniform(steps);
    r.cross = uniform((int)__any((lane & 15) == 0 && f < lane)) != 0;
    const int lr = lane & 15, row = lane >> 4;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
        const int d = 1 << s2;
        r.m[s2] = (lr >= d && lane - d >= f) ? 1.f : 0.f;
    }
    r.m[4] = ((row == 1 || row == 3) && 16 * row - 1 >= f) ? 1.f : 0.f;
    r.m[5] = ((row == 2 || row == 3) && 31 >= f) ? 1.f : 0.f;
    return r;
}

// The same segmented scan on two values.
#define ND_SEG_STEP2(x, y, m, DPP)                              \
    asm volatile("s_nop 1\n\t"                                 \
                 "v_fmac_f32_dpp %0, %0, %2 " DPP "\n\t"        \
                 "v_fmac_f32_dpp %1, %1, %2 " DPP                \
                 : "+v"(x), "+v"(y)                              \
                 : "v"(m))
__device__ __forceinline__ void seg_scan2(float& x, float& y, const Runs& r) {
    if (r.nsteps > 0) ND_SEG_STEP2(x, y, r.m[0], "row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    if (r.nsteps > 1) ND_SEG_STEP2(x, y, r.m[1], "row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    if (r.nsteps > 2) ND_SEG_STEP2(x, y, r.m[2], "row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    if (r.nsteps > 3) ND_SEG_STEP2(x, y, r.m[3], "row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    if (r.cross) {
        ND_SEG_STEP2(x, y, r.m[4], "row_bcast:15 row_mask:0xa bank_mask:0xf");
        ND_SEG_STEP2(x, y, r.m[5], "row_bcast:31 row_mask:0xc bank_mask:0xf");
    }
}

// A contracted row R = sum_h Nv_h Pw in the tile's frame translated by c:
// Pw - c w, i.e. (R_xyz - c R_w, R_w).  The backward works in this frame so
// that its sums of -(g . S)/W carry |S - c| (the tile's extent) instead of
// |S|; dL/dw, the small difference P . dL/dPw_xyz + dL/dPw_w of two such
// sums, then keeps its FP32 accuracy on nets far from the origin.
template <class St>
__device__ __forceinline__ float4 center4(float4 R, const St& st) {
    return make_float4(__builtin_fmaf(-st.cx, R.w, R.x), __builtin_fmaf(-st.cy, R.w, R.y),
                       __builtin_fmaf(-st.cz, R.w, R.z), R.w);
}

// Flush control row i (accumulator G) of the tile: the dV partial, and G
// itself into the slot's gacc row i - i0 for the gather pass.  Row i is
// staged in the block (or read from global).
template <int QM, bool BLK>
__device__ __forceinline__ void flush_row(const Surf& s, BwdState<QM>& st, const Block& bk, int i, int i0,
                                          float4 G, float4* __restrict__ gacc, bool want_pw, bool want_kv) {
    const int lane = lane_opaque();
    const int q = st.q;
    if (want_kv) {
        // (Pw - c w) . G = Pw . G - w (c . G_xyz)
        const float cg = __builtin_fmaf(st.cx, G.x, __builtin_fmaf(st.cy, G.y, st.cz * G.z));
        if constexpr (BLK) {
            const float4* row = block_row(bk, i, st.jb);
#pragma unroll
            for (int h = 0; h <= QM; ++h)
                if (h <= q) {
                    const float4 pw = row[h];
                    st.f[h] += __builtin_fmaf(-pw.w, cg, dot4(pw, G));
                }
        } else {
#pragma unroll
            for (int h = 0; h <= QM; ++h)
                if (h <= q) {
                    const float4 pw = load_pw(s, i, st.jb + h);
                    st.f[h] += __builtin_fmaf(-pw.w, cg, dot4(pw, G));
                }
        }
    }
    // inactive columns hold G = 0 (their dL/dS is zero), so the row is stored whole
    if (want_pw) gacc[(size_t)(i - i0) * kWave + lane] = G;
}

// Column set-up of a backward tile (independent of the degree in u): the
// lane's v-span and basis, and the tile's control-column range.
template <int QM, bool TAB = false>
__device__ __forceinline__ void bwd_columns(const Surf& s, int q, int col0, float vb, BwdState<QM>& st,
                                            const ColPre<QM>* pre = nullptr) {
    st.q = q;
    int j0, ncols;
    st.kb = tile_columns<QM, TAB>(s, q, col0, vb, st.Nv, st.act, j0, ncols, pre);
    st.jb = st.kb - q;
#pragma unroll
    for (int h = 0; h <= QM; ++h) st.f[h] = 0.f;
    st.j0 = j0;
    st.ncols = ncols;
}

// One tile of the gather as its wave sees it: slot, offsets of the column
// table and of gacc in it, degree in v.
struct GatTile {
    char* slot;
    size_t ctab_off, gacc_off;
    int q;
};

// A tile's header and this lane's column-table entry, loaded a tile ahead.
template <int QM>
struct GatPre {
    int4 hd;
    int first;
    float nv[QM + 1];
};

template <int QM>
__device__ __forceinline__ void gat_prefetch(const GatTile& t, GatPre<QM>& p) {
    const int lane = lane_id();
    p.hd = *reinterpret_cast<const int4*>(t.slot);
    const int* ct = reinterpret_cast<const int*>(t.slot + t.ctab_off);
    p.first = ct[lane];
    const float* cn = reinterpret_cast<const float*>(ct + kWave) + lane * (t.q + 1);
#pragma unroll
    for (int h = 0; h <= QM; ++h) p.nv[h] = h <= t.q ? cn[h] : 0.f;
}

// The gather, by one workgroup: tiles k = blockIdx, blockIdx + gridDim, ...
// of the source's order; within a tile, wave w takes the blocks w,
// w + kWavesPerWG, ... (column block outer), so a tile with many blocks is
// spread over the workgroup's waves.  For each tile, control rows i0..i1 and
// control columns j0..j1 (slot header):
//   rect[i - i0][jj] = sum_b M[jj][b] G_i(b),   M[jj][b] = Nv_{jj-first(b)}(v_b)
// (zero outside 0..q; inactive columns b have G = 0), the v-contraction of
// the flushed accumulators, with first(b) and Nv from the column table the
// row loop wrote.  Per tile a small banded matrix product, (ncols x 64) by
// (64 x 4 values per control row), computed with FP32 MFMA
// (v_mfma_f32_16x16x4f32): blocks of 16 control columns by 16 values (four
// control rows of G's four components), 64 samples in 16 steps of 4.
// Operand layout of that instruction on a wave64 (lane l): A[l%16][l/16],
// B[l/16][l%16], D[4(l/16)+v][l%16] for v = 0..3.  Latency is hidden in
// software: each wave loads the next tile's record, header and table while
// the current tile runs, and its next block's G values while the current
// block is multiplied.  Each output value is one block's fixed sequence of
// MFMAs: deterministic, and independent of which wave ran it.  Src supplies
// fetch(k) (a raw tile record, loaded ahead) and unpack(raw, k).
template <int QM, class Src>
__device__ __forceinline__ void gather_tiles(int ntiles, const Src& src, GatTab<QM>* tab) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x / kWave));
    const int lm = lane & 15, lk = lane >> 4;  // A row / B column; A column / B row (sample within a step)
    const int rr = lm >> 2, cc = lm & 3;       // B column lm = (control row rr of the block, component cc)
    const int G = (int)gridDim.x;
    int k = (int)blockIdx.x;
    if (k >= ntiles) return;
    GatTile cur = src.unpack(src.fetch(k), k);
    auto raw = src.fetch(k + G < ntiles ? k + G : k);
    GatPre<QM> pc;
    gat_prefetch<QM>(cur, pc);
    for (;;) {
        // this tile's table into the wave's LDS (the previous tile's reads of
        // it came first: one wave, LDS in order)
        tab->first[lane] = pc.first;
#pragma unroll
        for (int h = 0; h <= QM; ++h) tab->nv[lane * (QM + 1) + h] = pc.nv[h];
        wave_lds_sync();
        const int nrows = uniform(pc.hd.y - pc.hd.x + 1), ncols = uniform(pc.hd.w - pc.hd.z + 1);
        const int q = cur.q;
        const float* gacc = reinterpret_cast<const float*>(cur.slot + cur.gacc_off);
        float* rect = reinterpret_cast<float*>(cur.slot + kSlotHead);
        // the next tile: its record was loaded a tile ago; load the one after
        // it, and the next tile's header and table
        const int kn = k + G;
        GatTile nxt = cur;
        GatPre<QM> pn = pc;
        if (kn < ntiles) {
            nxt = src.unpack(raw, kn);
            raw = src.fetch(kn + G < ntiles ? kn + G : kn);
            gat_prefetch<QM>(nxt, pn);
        }
        // B operands of row block g: G_{4g + rr}(4 s4 + lk).cc (inactive
        // columns hold zeros).  A row past the last is read as the last row:
        // written data, reaching only output columns that are not stored, so
        // no load is predicated and all 16 are in flight at once.
        const int rlast = nrows - 1;
        auto load_b = [&](int g, float B[16]) {
            const float* src_row = gacc + ((size_t)min(4 * g + rr, rlast) * kWave + lk) * 4 + cc;
#pragma unroll
            for (int s4 = 0; s4 < 16; ++s4) B[s4] = src_row[s4 * 16];
        };
        const int ngr = (nrows + 3) >> 2, nmb = (ncols + 15) >> 4;
        const int npairs = ngr * nmb;
        if (wv < npairs) {
            float Bc[16];
            load_b(wv % ngr, Bc);
            float A[16];
            int amb = -1;
            for (int pidx = wv; pidx < npairs; pidx += kWavesPerWG) {
                const int mb = pidx / ngr, g = pidx - mb * ngr;
                const int pn2 = pidx + kWavesPerWG;
                float Bn[16];
                if (pn2 < npairs) load_b(pn2 % ngr, Bn);
                if (mb != amb) {
                    // A: M[16 mb + lm][4 s4 + lk] for the 16 steps; all table
                    // reads independent (clamped index, times a 0/1 mask; the
                    // table holds finite values for every column)
                    amb = mb;
                    int off[16];
#pragma unroll
                    for (int s4 = 0; s4 < 16; ++s4) off[s4] = 16 * mb + lm - tab->first[4 * s4 + lk];
#pragma unroll
                    for (int s4 = 0; s4 < 16; ++s4) {
                        const float x = tab->nv[(4 * s4 + lk) * (QM + 1) + min(max(off[s4], 0), QM)];
                        A[s4] = x * ((off[s4] >= 0 && off[s4] <= q) ? 1.f : 0.f);
                    }
                }
                f4v D = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s4 = 0; s4 < 16; ++s4)
                    D = __builtin_amdgcn_mfma_f32_16x16x4f32(A[s4], Bc[s4], D, 0, 0, 0);
                const int row = 4 * g + rr;
                if (row < nrows) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int jj = 16 * mb + 4 * lk + v;
                        if (jj < ncols) rect[((size_t)row * ncols + jj) * 4 + cc] = D[v];
                    }
                }
#pragma unroll
                for (int s4 = 0; s4 < 16; ++s4) Bc[s4] = Bn[s4];
            }
        }
        if (kn >= ntiles) break;
        k = kn;
        cur = nxt;
        pc = pn;
        wave_lds_sync();
    }
}

// Finish a batch of nb rows of dL/dNu: add the four 16-lane partials of
// each (row, r) in a fixed order and store them contiguously.
template <int P>
__device__ __forceinline__ void flush_e(BwdLds* L, int nb, float* __restrict__ e_out) {
    const int lane = lane_opaque();
    wave_lds_sync();
    for (int idx = lane; idx < nb * (P + 1); idx += kWave) {
        const int t = idx / (P + 1), r = idx - t * (P + 1);
        const float* e = L->ebuf + (t * 4) * (P + 1) + r;
        e_out[idx] = ((e[0] + e[P + 1]) + e[2 * (P + 1)]) + e[3 * (P + 1)];
    }
    wave_lds_sync();
}

// dL/dS of row a for this lane's column (zero on inactive lanes)
__device__ __forceinline__ float3 load_g(const float* __restrict__ gpts, int a, int nv_s, int b, bool act) {
    float3 v = make_float3(0.f, 0.f, 0.f);
    if (act) {
        const float* gp = gpts + 3 * ((size_t)a * nv_s + b);
        v = make_float3(gp[0], gp[1], gp[2]);
    }
    return v;
}

template <int P, int QM, bool BLK, bool TAB = false>
__device__ __forceinline__ void bwd_rows_impl(const Surf& s, BwdState<QM>& st, Block& bk, int col0, int row0,
                                              int row1, float u0, const float* __restrict__ gpts, SlotView out,
                                              BwdLds* L, unsigned mask, const RowPre<P>* rpre = nullptr) {
    const int lane = lane_id();
    const bool want_pw = (mask & 3u) != 0;
    const bool want_ku = (mask & 4u) != 0;
    const bool want_kv = (mask & 8u) != 0;
    const int q = st.q;
    const int b = col0 + lane;
    if (want_pw) {
        // the gather's column table: this column's first control column and basis
        out.ctab[lane] = st.act ? st.jb - st.j0 : kGatherOff;
        float* nv = reinterpret_cast<float*>(out.ctab + kWave) + lane * (q + 1);
#pragma unroll
        for (int h = 0; h <= QM; ++h)
            if (h <= q) nv[h] = st.Nv[h];
    }
    float4 R[P + 1], G[P + 1];
    int cur = -1, i0 = 0;
    // dL/dS is loaded one row ahead of its use, straight into registers
    float3 gn = load_g(gpts, row0, s.nv_s, b, st.act);
    for (int a0 = row0; a0 < row1; a0 += kWave) {
        const int nr = min(kWave, row1 - a0);
        float Nu_l[P + 1];
        const float ua = TAB ? 0.f : (a0 == row0 ? u0 : s.us[a0 + min(lane, nr - 1)]);
        const int ka_l = row_basis<P, TAB>(s, a0, nr, ua, Nu_l, a0 == row0 ? rpre : nullptr);
        int eb = 0;  // rows in the current dL/dNu batch
        for (int t = 0; t < nr; ++t) {
            const float3 g = gn;
            if (a0 + t + 1 < row1) gn = load_g(gpts, a0 + t + 1, s.nv_s, b, st.act);
            const int ka = bcast_lane(ka_l, t);
            if (cur < 0) {
                cur = ka;
                i0 = ka - P;
                ensure_rows<BLK>(s, bk, ka - P, ka);
                {   // frame origin: the control point in the middle of the first window
                    const int ic = ka - P + P / 2, jc = st.j0 + (st.ncols - 1) / 2;
                    float4 pc;
                    if constexpr (BLK) pc = *block_row(bk, ic, jc);
                    else pc = load_pw(s, ic, jc);
                    const float rw = recip(pc.w);
                    st.cx = uniform_f(pc.x * rw);
                    st.cy = uniform_f(pc.y * rw);
                    st.cz = uniform_f(pc.z * rw);
                }
#pragma unroll
                for (int r = 0; r <= P; ++r) {
                    R[r] = center4(blk_contract<QM, BLK>(s, bk, ka - P + r, st.jb, st.Nv, q), st);
                    G[r] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
            } else {
                // rows are non-decreasing, so the window only moves forward;
                // each control row leaving it is flushed
                while (cur < ka) {
                    flush_row<QM, BLK>(s, st, bk, cur - P, i0, G[0], out.gacc, want_pw, want_kv);
#pragma unroll
                    for (int r = 0; r < P; ++r) {
                        R[r] = R[r + 1];
                        G[r] = G[r + 1];
                    }
                    ++cur;
                    G[P] = make_float4(0.f, 0.f, 0.f, 0.f);
                    ensure_rows<BLK>(s, bk, cur - P, cur);
                    R[P] = center4(blk_contract<QM, BLK>(s, bk, cur, st.jb, st.Nv, q), st);
                }
            }
            float Nu[P + 1];
#pragma unroll
            for (int r = 0; r <= P; ++r) Nu[r] = bcast_lane(Nu_l[r], t);
            // recompute S' (nothing is saved by the forward)
            float4 sp = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int r = 0; r <= P; ++r) sp = fma4(Nu[r], R[r], sp);
            const float rw = recip_fast(sp.w);
            const float cx = g.x * rw, cy = g.y * rw, cz = g.z * rw;
            const float cw = -(cx * sp.x + cy * sp.y + cz * sp.z) * rw;
            const float4 hv = make_float4(cx, cy, cz, cw);
#pragma unroll
            for (int r = 0; r <= P; ++r) G[r] = fma4(Nu[r], hv, G[r]);
            if (want_ku) {
                float e[P + 1];
#pragma unroll
                for (int r = 0; r <= P; ++r) e[r] = dot4(R[r], hv);
                row16_sum_n(e);
                if ((lane & 15) == 0) {
                    float* dst = L->ebuf + (eb * 4 + (lane >> 4)) * (P + 1);
#pragma unroll
                    for (int r = 0; r <= P; ++r) dst[r] = e[r];
                }
                if (++eb == kEBatch) {
                    flush_e<P>(L, eb, out.e + (size_t)(a0 + t + 1 - eb - row0) * (P + 1));
                    eb = 0;
                }
            }
        }
        if (want_ku && eb > 0) flush_e<P>(L, eb, out.e + (size_t)(a0 + nr - eb - row0) * (P + 1));
    }
    // flush the rows still in the window (all still staged)
    const int i1 = cur;
    for (int r = 0; r <= P; ++r) {
        flush_row<QM, BLK>(s, st, bk, cur - P, i0, G[0], out.gacc, want_pw, want_kv);
#pragma unroll
        for (int m = 0; m < P; ++m) G[m] = G[m + 1];
        ++cur;
    }

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
        *out.center = make_float4(st.cx, st.cy, st.cz, 0.f);
    }
}

template <int P, int QM, bool TAB = false>
__device__ __forceinline__ void bwd_rows(const Surf& s, BwdState<QM>& st, int col0, int row0, int row1, float u0,
                                         const float* __restrict__ gpts, SlotView out, BwdLds* L,
                                         unsigned mask, const RowPre<P>* rpre = nullptr) {
    Block bk = make_block(L->blk, st.j0, st.ncols, P);
    if (bk.on)
        bwd_rows_impl<P, QM, true, TAB>(s, st, bk, col0, row0, row1, u0, gpts, out, L, mask, rpre);
    else
        bwd_rows_impl<P, QM, false, TAB>(s, st, bk, col0, row0, row1, u0, gpts, out, L, mask, rpre);
}

// Stage the tile's first inputs (knots into LDS); returns the surface view
// that reads the knots from LDS.
__device__ __forceinline__ Surf bwd_stage(const Surf& sg, int p, int q, int col0, int row0, int row1, BwdLds* L,
                                          TileIn& in) {
    Surf s = sg;
    in = stage_tile(sg, p, q, col0, row0, row1, L->knots[0], L->knots[1]);
    s.ku = L->knots[0];
    s.kv = L->knots[1];
    return s;
}

template <int P, int QM, bool TAB = false>
__device__ __forceinline__ void bwd_tile(const Surf& sg, int q, int col0, int row0, int row1,
                                         const float* __restrict__ gpts, SlotView out, BwdLds* L, unsigned mask) {
    TileIn in;
    ColPre<QM> cpre;
    RowPre<P> rpre;
    if constexpr (TAB) {
        col_prefetch<QM>(sg, q, col0, cpre);
        row_prefetch<P>(sg, row0, row1, rpre);
    }
    const Surf s = bwd_stage(sg, P, q, col0, row0, row1, L, in);
    BwdState<QM> st;
    bwd_columns<QM, TAB>(s, q, col0, in.v, st, &cpre);
    bwd_rows<P, QM, TAB>(s, st, col0, row0, row1, in.u0, gpts, out, L, mask, &rpre);
}

// --------------------------------------------------------------------------
// finalize: one wave per surface (kWavesPerWG surfaces per workgroup)
// --------------------------------------------------------------------------
constexpr int kFinMaxTiles = 64;  // tile headers staged in LDS (more: read from global)
constexpr int kFinCp = 4;         // control points per lane per pass (registers for six waves/SIMD)
constexpr int kFinW = 2 * kMaxDeg + 2;

struct FinLds {
    float knots[kWG];
    int4 hdr[kFinMaxTiles];
    float contrib[kWave * kFinW];  // per run head of the chunk, run sums of the knot-window adjoints
    short head_of[kWG];            // span - first span of the chunk -> head lane, or -1
};

// Tiles of one surface in natural order (row blocks outer, 64-column blocks
// inner): slot pointer, column start and row range of tile t.
struct TileRef {
    const char* slot;
    int col0, row0, row1;
    int alloc_rows;  // rows the slot was sized for (>= row1 - row0)
};

// Tile i of a surface whose equal-sized slots start at slot0 (pure
// arithmetic: no table read on the finalize's dependent-load chains).
__device__ __forceinline__ TileRef surface_tile(const char* slot0, size_t stride, int i, int ncb, int rows,
                                                int nu_s) {
    TileRef tr;
    const int rb = i / ncb, cb = i - rb * ncb;
    tr.slot = slot0 + (size_t)i * stride;
    tr.col0 = cb * kWave;
    tr.row0 = rb * rows;
    tr.row1 = min(nu_s, tr.row0 + rows);
    tr.alloc_rows = rows;
    return tr;
}

// Knot gradient of one direction: for every sample x_a of the direction,
// coef(a)[r] = dL/dN_{k_a-D+r}(x_a) is turned into per-knot adjoints
// g_t(a) = d/dU_{k_a-D+t} by basis_knot_adjoint (t = 0..2D+1).  Samples come
// 64 at a time; within a chunk, the samples of one span form a run of lanes
// (spans are non-decreasing), so each g_t is first summed over its run by a
// DPP segmented scan.  Knot kk then takes, for each t, the run sum of the
// span kk + D - t (one LDS read through the run-head table), accumulating
// in FP64 in a fixed order (chunks, then t).
template <int D, class CoefAt>
__device__ __forceinline__ void knot_gradient(const float* __restrict__ Ug, int nc, const float* __restrict__ xs,
                                              int ns, CoefAt coef_at, float* __restrict__ gout, FinLds* L) {
    constexpr int W = 2 * D + 2;
    const int lane = lane_id();
    const int nk = nc + D + 1;
    const int n = nc - 1;
    wave_lds_sync();
    for (int i = lane; i < nk; i += kWave) L->knots[i] = Ug[i];
    wave_lds_sync();
    const float* U = L->knots;
    double acc[kWG / kWave];
#pragma unroll
    for (int m = 0; m < kWG / kWave; ++m) acc[m] = 0.0;
    for (int g0 = 0; g0 < ns; g0 += kWG) {
        // the parameters of four chunks are fetched together, and each chunk's
        // coefficients while the previous chunk is being worked on
        float xv[kWG / kWave];
#pragma unroll
        for (int c = 0; c < kWG / kWave; ++c) xv[c] = xs[min(g0 + c * kWave + lane, ns - 1)];
        float en[D + 1];
        coef_at(min(g0 + lane, ns - 1), en);
#pragma unroll
        for (int c = 0; c < kWG / kWave; ++c) {
            const int a0 = g0 + c * kWave;
            if (a0 >= ns) break;
            const int a = a0 + lane;
            const int cnt = min(kWave, ns - a0);
            const bool valid = a < ns;
            float e[D + 1];
#pragma unroll
            for (int r = 0; r <= D; ++r) e[r] = en[r];
            if (c + 1 < kWG / kWave && a0 + kWave < ns) coef_at(min(a + kWave, ns - 1), en);
            int k = 0;
            float g[W];
#pragma unroll
            for (int t = 0; t < W; ++t) g[t] = 0.0f;
            if (valid) {
                const float x = clamp_param(U, D, n, xv[c]);
                k = find_span(U, D, n, x);
                basis_knot_adjoint<D>(U, k, x, e, g);
            }
            const int kfirst = bcast_lane(k, 0);
            const int nkeys = bcast_lane(k, cnt - 1) - kfirst + 1;
            // lanes past the last sample get keys of their own (runs of one, adding zeros)
            const int key = valid ? k - kfirst : 0x40000000 + lane;
            const Runs rr = wave_runs(key);
            // W = 2D is even: four values per scan while they last, then two
#pragma unroll
            for (int t = 0; t + 3 < W; t += 4) {
                float4 x = make_float4(g[t], g[t + 1], g[t + 2], g[t + 3]);
                seg_scan4(x, rr);
                g[t] = x.x;
                g[t + 1] = x.y;
                g[t + 2] = x.z;
                g[t + 3] = x.w;
            }
            if constexpr (W % 4 != 0) seg_scan2(g[W - 2], g[W - 1], rr);
            for (int o = lane; o < nkeys; o += kWave) L->head_of[o] = (short)-1;
            wave_lds_sync();
            if (valid && rr.head) {
                L->head_of[key] = (short)lane;
#pragma unroll
                for (int t = 0; t < W; ++t) L->contrib[lane * W + t] = g[t];
            }
            wave_lds_sync();
#pragma unroll
            for (int m = 0; m < kWG / kWave; ++m) {
                if (m * kWave >= nk) break;
                const int kk = lane + m * kWave;
                if (kk < nk) {
#pragma unroll
                    for (int t = 0; t < W; ++t) {
                        const int o = kk + D - t - kfirst;
                        const int hl = (o >= 0 && o < nkeys) ? (int)L->head_of[o] : -1;
                        if (hl >= 0) acc[m] += (double)L->contrib[hl * W + t];
                    }
                }
            }
            wave_lds_sync();
        }
    }
#pragma unroll
    for (int m = 0; m < kWG / kWave; ++m) {
        const int kk = lane + m * kWave;
        if (kk < nk) gout[kk] = (float)acc[m];
    }
}

// Finalize work of one surface, in parts that can run on different waves:
//   kFinPW + c : dL/dP, dL/dw of control points [c * kFinChunk, (c + 1) * kFinChunk)
//   kFinKU     : dL/dU;   kFinKV : dL/dV.
constexpr int kFinChunk = kWave * kFinCp;  // control points per dP/dW part
constexpr int kFinKU = 0, kFinKV = 1, kFinPW = 2;

// Sum of the tile rectangles over this lane's control points of one chunk,
// tiles in fixed order, two tiles' loads in flight at a time.
template <class TileAt>
__device__ __forceinline__ void fin_pw_chunk(const Surf& s, int ntiles, TileAt tile_at, int chunk,
                                             float* __restrict__ gctrl, float* __restrict__ gw, unsigned mask,
                                             FinLds* L) {
    const int lane = lane_id();
    const bool hdr_lds = ntiles <= kFinMaxTiles;
    if (hdr_lds)
        for (int t = lane; t < ntiles; t += kWave) L->hdr[t] = *reinterpret_cast<const int4*>(tile_at(t).slot);
    wave_lds_sync();
    const int ncp = s.nu_c * s.nv_c;
    const int base = chunk * kFinChunk;
    float4 acc[kFinCp];
    int ii[kFinCp], jj[kFinCp];
#pragma unroll
    for (int c = 0; c < kFinCp; ++c) {
        acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
        const int ij = base + c * kWave + lane;
        ii[c] = ij / s.nv_c;
        jj[c] = ij - ii[c] * s.nv_c;
    }
    // v: the tile's rect entries; c: its frame origin.  The header comes from
    // LDS or from the slot, in two compiled paths (one path with a run-time
    // choice let the compiler merge both into generic-address loads).
    auto load_tile = [&](auto hl, int t, float4 v[kFinCp], float4& c) {
        const char* slot = tile_at(t).slot;
        c = *reinterpret_cast<const float4*>(slot + 16);
        int4 h;
        if constexpr (decltype(hl)::value) h = L->hdr[t];
        else h = *reinterpret_cast<const int4*>(slot);
        const float4* rect = reinterpret_cast<const float4*>(slot + kSlotHead);
        const int pitch = h.w - h.z + 1;
#pragma unroll
        for (int c = 0; c < kFinCp; ++c) {
            const int ij = base + c * kWave + lane;
            const bool in = ij < ncp && ii[c] >= h.x && ii[c] <= h.y && jj[c] >= h.z && jj[c] <= h.w;
            v[c] = in ? rect[(size_t)(ii[c] - h.x) * pitch + (jj[c] - h.z)] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    // acc.w collects dL/dw - P . dL/dPw_xyz: the tile's rect w (its frame's
    // dL/dw - (P - c) . dL/dPw_xyz) minus c . dL/dPw_xyz
    auto add = [&](const float4 v[kFinCp], const float4 ct) {
#pragma unroll
        for (int c = 0; c < kFinCp; ++c) {
            acc[c].x += v[c].x;
            acc[c].y += v[c].y;
            acc[c].z += v[c].z;
            acc[c].w += v[c].w - (ct.x * v[c].x + ct.y * v[c].y + ct.z * v[c].z);
        }
    };
    // two tiles' loads in flight at a time; sums still in tile order
    auto sum_tiles = [&](auto hl) {
        int t = 0;
        for (; t + 1 < ntiles; t += 2) {
            float4 va[kFinCp], vb[kFinCp], ca, cb;
            load_tile(hl, t, va, ca);
            load_tile(hl, t + 1, vb, cb);
            add(va, ca);
            add(vb, cb);
        }
        if (t < ntiles) {
            float4 va[kFinCp], ca;
            load_tile(hl, t, va, ca);
            add(va, ca);
        }
    };
    if (hdr_lds) sum_tiles(std::true_type{});
    else sum_tiles(std::false_type{});
#pragma unroll
    for (int c = 0; c < kFinCp; ++c) {
        const int ij = base + c * kWave + lane;
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

// dL/dU: e(a) = sum over the column blocks of a's row block.
template <int P, class TileAt>
__device__ __forceinline__ void fin_knots_u(const Surf& s, int ntiles, TileAt tile_at, float* __restrict__ gku,
                                            FinLds* L) {
    const size_t rect_bytes = 16 * (size_t)s.nu_c * s.nv_c;
    const int ncb = (s.nv_s + kWave - 1) / kWave;
    const int rows = ntiles > 0 ? tile_at(0).alloc_rows : 1;
    auto coef = [&](int a, float e[P + 1]) {
#pragma unroll
        for (int r = 0; r <= P; ++r) e[r] = 0.0f;
        const int rb = a / rows;
        for (int cb = 0; cb < ncb; ++cb) {
            const TileRef tr = tile_at(rb * ncb + cb);
            const float* ev = reinterpret_cast<const float*>(tr.slot + kSlotHead + rect_bytes) +
                              (size_t)(a - tr.row0) * (P + 1);
#pragma unroll
            for (int r = 0; r <= P; ++r) e[r] += ev[r];
        }
    };
    knot_gradient<P>(s.ku, s.nu_c, s.us, s.nu_s, coef, gku, L);
}

// dL/dV: f(b) = sum over the row blocks of b's column block (p, the degree
// in u, only places f inside the slot).
template <int Q, class TileAt>
__device__ __forceinline__ void fin_knots_v(const Surf& s, int ntiles, TileAt tile_at, int p,
                                            float* __restrict__ gkv, FinLds* L) {
    const size_t rect_bytes = 16 * (size_t)s.nu_c * s.nv_c;
    const int ncb = (s.nv_s + kWave - 1) / kWave;
    const int nrb = ncb > 0 ? ntiles / ncb : 0;
    auto coef = [&](int b, float f[Q + 1]) {
#pragma unroll
        for (int h = 0; h <= Q; ++h) f[h] = 0.0f;
        const int cb = b / kWave;
        for (int rb = 0; rb < nrb; ++rb) {
            const TileRef tr = tile_at(rb * ncb + cb);
            const float* fv = reinterpret_cast<const float*>(
                tr.slot + kSlotHead + rect_bytes + align16(sizeof(float) * (size_t)tr.alloc_rows * (p + 1)));
#pragma unroll
            for (int h = 0; h <= Q; ++h) f[h] += fv[(b - tr.col0) * (Q + 1) + h];
        }
    };
    knot_gradient<Q>(s.kv, s.nv_c, s.vs, s.nv_s, coef, gkv, L);
}

// One finalize part (see kFinPW / kFinKU / kFinKV); the knot parts are
// compiled per degree of their own direction only.
template <int DM, class TileAt>
__device__ __forceinline__ void finalize_part(const Surf& s, int ntiles, TileAt tile_at, int p, int q, int part,
                                              float* __restrict__ gctrl, float* __restrict__ gw,
                                              float* __restrict__ gku, float* __restrict__ gkv, unsigned mask,
                                              FinLds* L) {
    if (part >= kFinPW) {
        if (mask & 3u) fin_pw_chunk(s, ntiles, tile_at, part - kFinPW, gctrl, gw, mask, L);
    } else if (part == kFinKU) {
        if (!(mask & 4u)) return;
        switch (p) {
#define ND_KU(D) \
    case D:      \
        if constexpr (D <= DM) fin_knots_u<D>(s, ntiles, tile_at, gku, L); \
        break;
            ND_KU(1) ND_KU(2) ND_KU(3) ND_KU(4) ND_KU(5) ND_KU(6) ND_KU(7)
#undef ND_KU
            default: break;
        }
    } else {
        if (!(mask & 8u)) return;
        switch (q) {
#define ND_KV(D) \
    case D:      \
        if constexpr (D <= DM) fin_knots_v<D>(s, ntiles, tile_at, p, gkv, L); \
        break;
            ND_KV(1) ND_KV(2) ND_KV(3) ND_KV(4) ND_KV(5) ND_KV(6) ND_KV(7)
#undef ND_KV
            default: break;
        }
    }
}

// The same with both degrees known at compile time (uniform batches).
template <int P, int Q, class TileAt>
__device__ __forceinline__ void finalize_part_pq(const Surf& s, int ntiles, TileAt tile_at, int part,
                                                 float* __restrict__ gctrl, float* __restrict__ gw,
                                                 float* __restrict__ gku, float* __restrict__ gkv, unsigned mask,
                                                 FinLds* L) {
    if (part >= kFinPW) {
        if (mask & 3u) fin_pw_chunk(s, ntiles, tile_at, part - kFinPW, gctrl, gw, mask, L);
    } else if (part == kFinKU) {
        if (mask & 4u) fin_knots_u<P>(s, ntiles, tile_at, gku, L);
    } else {
        if (mask & 8u) fin_knots_v<Q>(s, ntiles, tile_at, P, gkv, L);
    }
}

// Number of parts of a surface's finalize.
__host__ __device__ inline int fin_parts(int nu_c, int nv_c) {
    return kFinPW + (nu_c * nv_c + kFinChunk - 1) / kFinChunk;
}

// All parts of one surface on one wave (uniform batches).
template <int P, int Q, class TileAt>
__device__ __forceinline__ void finalize_surface(const Surf& s, int ntiles, TileAt tile_at, float* __restrict__ gctrl,
                                                 float* __restrict__ gw, float* __restrict__ gku,
                                                 float* __restrict__ gkv, unsigned mask, FinLds* L) {
    const int np = fin_parts(s.nu_c, s.nv_c);
    for (int part = 0; part < np; ++part) {
        finalize_part_pq<P, Q>(s, ntiles, tile_at, part, gctrl, gw, gku, gkv, mask, L);
        wave_lds_sync();
    }
}

// Surface s of a uniform batch (degrees p, q).
__device__ __forceinline__ Surf uniform_surf(const UniformArgs& a, int s, int p, int q) {
    Surf r;
    const size_t cp = (size_t)a.nu_c * a.nv_c;
    r.ctrl = a.ctrl + (size_t)s * cp * 3;
    r.w = a.w + (size_t)s * cp;
    r.ku = a.ku + (size_t)s * (a.nu_c + p + 1);
    r.kv = a.kv + (size_t)s * (a.nv_c + q + 1);
    r.us = a.us + (a.uv_shared ? 0 : (size_t)s * a.nu_s);
    r.vs = a.vs + (a.uv_shared ? 0 : (size_t)s * a.nv_s);
    r.nu_c = a.nu_c;
    r.nv_c = a.nv_c;
    r.nu_s = a.nu_s;
    r.nv_s = a.nv_s;
    r.tsu = nullptr;
    r.tbu = nullptr;
    r.tsv = nullptr;
    r.tbv = nullptr;
    if (a.tab_u) {  // fixed-knot tables: spans, then basis rows at the next 256-byte boundary
        const char* tu = a.tab_u + (size_t)s * a.tab_u_stride;
        const char* tv = a.tab_v + (size_t)s * a.tab_v_stride;
        r.tsu = reinterpret_cast<const int*>(tu);
        r.tbu = reinterpret_cast<const float*>(tu + basis_table_split(a.nu_s));
        r.tsv = reinterpret_cast<const int*>(tv);
        r.tbv = reinterpret_cast<const float*>(tv + basis_table_split(a.nv_s));
    }
    return r;
}

}  // namespace nd
