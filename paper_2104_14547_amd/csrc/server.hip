// Continuous-batching server of surface evaluation + gradient requests
// (native engine).  The surfaces stay resident on the device; a request
// brings a parameter grid (us, vs) and target points T and receives S on the
// grid and the gradients of L = sum ||S - T||^2 with respect to the
// surface's control points, weights and both knot vectors: the forward of
// Sec. 3.1 and the backward of Sec. 3.2 per request, batched over requests
// as a ragged plan.
//
// Threads: the caller's threads submit and wait; an engine thread forms
// batches, packs them into a slot's pinned host buffer and queues the copy
// up, the plan, the forward, dL/dS = 2 (S - T), the backward, the gather of
// each request's gradients and the copy back on the slot's stream; a
// completion thread waits for each launched slot's event, copies every
// request's block to the caller's output buffer and wakes the waiters.  No
// Python runs on the serving path.
#include "nurbsdiff.h"

#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

constexpr size_t kAlign = 256;
constexpr int kPendingState = 1;  // state of a request not finished yet (finished: NURBS_OK or an error code)
constexpr int kGroups = 4;        // gradient arrays: ctrl, w, ku, kv

size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

double now_s() {
    timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

// One contiguous run of floats: src offset, dst offset, length.  Runs are
// cut into pieces of at most kSegChunk floats, one workgroup each, so that a
// large request spreads over many workgroups.
struct Seg {
    int64_t src, dst, n;
};
constexpr int64_t kSegChunk = 16384;

int64_t seg_pieces(int64_t n) { return (n + kSegChunk - 1) / kSegChunk; }

// Appends the pieces of the run (src, dst, n) at `out`; returns the new end.
Seg* emit_run(Seg* out, int64_t src, int64_t dst, int64_t n) {
    for (int64_t o = 0; o < n; o += kSegChunk) *out++ = Seg{src + o, dst + o, std::min(kSegChunk, n - o)};
    return out;
}

// g[dst + i] = 2 (res[dst + i] - tgt[src + i]): the adjoint of the squared
// distance, at the offsets where the forward wrote the request's points.
__global__ void k_residual(const Seg* __restrict__ segs, const float* __restrict__ res,
                           const float* __restrict__ tgt, float* __restrict__ g) {
    const Seg s = segs[blockIdx.x];
    for (int64_t i = threadIdx.x; i < s.n; i += blockDim.x) g[s.dst + i] = 2.0f * (res[s.dst + i] - tgt[s.src + i]);
}

// dst[seg.dst + i] = src[seg.src + i]: a request's gradient blocks out of
// the pool-sized gradient arrays into its result block.
__global__ void k_copy_segs(const Seg* __restrict__ segs, const float* __restrict__ src, float* __restrict__ dst) {
    const Seg s = segs[blockIdx.x];
    for (int64_t i = threadIdx.x; i < s.n; i += blockDim.x) dst[s.dst + i] = src[s.src + i];
}

// A parallel-for over a few helper threads: run(n, fn) calls fn(i) for
// every i in [0, n) on the helpers and the calling thread and returns when
// all calls have returned.  Used for the per-request copies into and out of
// the pinned buffers, which one thread cannot keep up with (the output
// copies also take the first-touch page faults of the callers' arrays).
class CopyPool {
public:
    explicit CopyPool(int helpers) {
        for (int t = 0; t < helpers; ++t) th_.emplace_back([this] { work(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            quit_ = true;
        }
        cv_.notify_all();
        for (std::thread& t : th_) t.join();
    }
    void run(int n, const std::function<void(int)>& fn) {
        if (n <= 0) return;
        if (th_.empty() || n == 1) {
            for (int i = 0; i < n; ++i) fn(i);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(m_);
            job_ = &fn;
            n_ = n;
            next_.store(0);
            active_ = (int)th_.size();
            ++gen_;
        }
        cv_.notify_all();
        for (int i; (i = next_.fetch_add(1)) < n;) fn(i);
        std::unique_lock<std::mutex> lk(m_);
        done_.wait(lk, [&] { return active_ == 0; });
        job_ = nullptr;
    }

private:
    void work() {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)>* f;
            int n;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return quit_ || gen_ != seen; });
                if (quit_) return;
                seen = gen_;
                f = job_;
                n = n_;
            }
            for (int i; (i = next_.fetch_add(1)) < n;) (*f)(i);
            std::lock_guard<std::mutex> lk(m_);
            if (--active_ == 0) done_.notify_one();
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(int)>* job_ = nullptr;
    int n_ = 0, active_ = 0;
    std::atomic<int> next_{0};
    uint64_t gen_ = 0;
    bool quit_ = false;
};

constexpr int kCopyHelpers = 3;  // per copying thread (engine, completion)

struct Req {
    int64_t id = 0;
    int surf = 0, nu_s = 0, nv_s = 0;
    const float *us = nullptr, *vs = nullptr, *tgt = nullptr;
    float* out = nullptr;
    double t_arr = 0.0;
    size_t nbytes = 0, ws = 0, tb = 0;  // device bytes in a batch; plan workspace and tables alone
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    char* arena = nullptr;   // device
    char* host = nullptr;    // pinned mirror of the arena's copied regions
    float* gflat = nullptr;  // device, the four pool-sized gradient arrays back to back
    std::vector<Req> batch;
    std::vector<nurbs_desc> desc;
    std::vector<int64_t> res_off;  // float offset of each request's result block
    std::vector<int64_t> tgt_off;  // float offset of each request's targets
    nurbs_plan* plan = nullptr;
    size_t res_o = 0;  // byte offset of the result region
    int rc = NURBS_OK;
    bool busy = false;
};

// The batch-formation rule, on any sequence of (surface, bytes) in arrival
// order: take requests while the batch's bytes fit `capacity` (with `fixed`
// bytes per batch) and fewer than `max_requests` are taken; a request for a
// surface already taken is passed over and stays queued; stop at the first
// request that does not fit, so it is not overtaken; look at most
// 4 * max_requests requests past the last one taken.
template <class SurfAt, class BytesAt>
void admit(int n, SurfAt surf_at, BytesAt bytes_at, size_t capacity, size_t fixed, int max_requests,
           std::vector<int>& take) {
    take.clear();
    size_t used = fixed;
    std::unordered_map<int, char> seen;
    int passed = 0;
    for (int i = 0; i < n && (int)take.size() < max_requests; ++i) {
        const int sf = surf_at(i);
        if (seen.count(sf)) {
            if (++passed > 4 * max_requests) break;
            continue;
        }
        const size_t b = bytes_at(i);
        if (used + b > capacity) break;
        used += b;
        seen[sf] = 1;
        take.push_back(i);
    }
}

}  // namespace

struct nurbs_server {
    int device = 0;
    nurbs_ctx* ctx = nullptr;   // the engine thread's
    nurbs_ctx* qctx = nullptr;  // plan size queries at submission (under qmu)
    std::vector<nurbs_desc> pool;
    const float *ctrl = nullptr, *w = nullptr, *ku = nullptr, *kv = nullptr;
    size_t gbase[kGroups] = {0, 0, 0, 0};  // float offsets of the gradient arrays in gflat
    size_t gtotal = 0;
    size_t slot_bytes = 0, fixed = 0;
    int max_req = 1;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_eng, cv_fin, cv_done;
    std::deque<Req> pending;
    std::deque<int> launched;  // slots in launch order
    std::vector<int> state;    // per request id
    std::vector<double> lat;
    int64_t low = 0;  // every id below has finished
    int64_t batches = 0, completed = 0;
    double eng_busy = 0.0, fin_busy = 0.0;  // seconds the two threads spent on batches
    bool stop = false, eng_done = false;
    std::string err;
    std::thread eng, fin;
    CopyPool pack{kCopyHelpers}, unpack{kCopyHelpers};

    std::mutex qmu;
    std::unordered_map<uint64_t, std::array<size_t, 2>> sizes;  // (surf, nu_s, nv_s) -> plan ws, tables
};

namespace {

int64_t grad_count(const nurbs_desc& d, int k) {
    switch (k) {
        case 0: return 3ll * d.nu_c * d.nv_c;
        case 1: return (int64_t)d.nu_c * d.nv_c;
        case 2: return d.nu_c + d.p + 1;
        default: return d.nv_c + d.q + 1;
    }
}
int64_t grad_off(const nurbs_desc& d, int k) {
    return k == 0 ? d.ctrl_off : k == 1 ? d.w_off : k == 2 ? d.ku_off : d.kv_off;
}
int64_t out_floats(const nurbs_desc& d, int nu_s, int nv_s) {
    int64_t n = 3ll * nu_s * nv_s;
    for (int k = 0; k < kGroups; ++k) n += grad_count(d, k);
    return n;
}
// segment records of a request: its residual pieces, its gradient pieces
int64_t residual_segs(int nu_s, int nv_s) { return seg_pieces(3ll * nu_s * nv_s); }
int64_t gather_segs(const nurbs_desc& d) {
    int64_t n = 0;
    for (int k = 0; k < kGroups; ++k) n += seg_pieces(grad_count(d, k));
    return n;
}

void set_err(nurbs_server* s, const std::string& m) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->err = m;
}

int hip_err(nurbs_server* s, hipError_t e, const char* what) {
    set_err(s, std::string(what) + ": " + hipGetErrorString(e));
    return NURBS_EDEVICE;
}

int plan_err(nurbs_server* s, nurbs_ctx* c, int rc, const char* what) {
    set_err(s, std::string(what) + ": " + nurbs_last_error(c));
    return rc;
}

// Packs `sl.batch` into the slot and queues its work on the slot's stream.
int launch(nurbs_server* s, Slot& sl) {
    const int n = (int)sl.batch.size();
    sl.res_off.resize(n);
    sl.tgt_off.resize(n);
    sl.desc.resize(n);
    size_t n_uv = 0, n_tgt = 0, n_res = 0, ws = NURBS_PLAN_WS_HEADER, tb = 0, nrs = 0, ngs = 0;
    for (int i = 0; i < n; ++i) {
        const Req& r = sl.batch[i];
        const size_t npts = (size_t)r.nu_s * r.nv_s;
        sl.res_off[i] = (int64_t)n_res;
        sl.tgt_off[i] = (int64_t)n_tgt;
        n_res += (size_t)out_floats(s->pool[r.surf], r.nu_s, r.nv_s);
        n_uv += (size_t)r.nu_s + r.nv_s;
        n_tgt += 3 * npts;
        ws += r.ws - NURBS_PLAN_WS_HEADER;
        tb += r.tb;
        nrs += (size_t)residual_segs(r.nu_s, r.nv_s);
        ngs += (size_t)gather_segs(s->pool[r.surf]);
    }
    const size_t nseg = nrs + ngs;
    const size_t o_tgt = al(4 * n_uv), o_seg = o_tgt + al(4 * n_tgt), o_res = o_seg + al(sizeof(Seg) * nseg);
    const size_t o_g = o_res + al(4 * n_res), o_ws = o_g + al(4 * n_res), o_tb = o_ws + al(ws);
    const size_t end = o_tb + al(tb);
    if (end > s->slot_bytes) {
        set_err(s, "batch exceeds the slot");
        return NURBS_EWORKSPACE;
    }
    // pack: parameters, targets, segment tables, descriptors
    float* huv = reinterpret_cast<float*>(sl.host);
    float* htgt = reinterpret_cast<float*>(sl.host + o_tgt);
    Seg* hseg = reinterpret_cast<Seg*>(sl.host + o_seg);
    Seg* rseg = hseg;        // residual pieces
    Seg* gseg = hseg + nrs;  // gradient pieces
    size_t cu = 0;
    for (int i = 0; i < n; ++i) {
        const Req& r = sl.batch[i];
        const nurbs_desc& pd = s->pool[r.surf];
        const size_t npts = (size_t)r.nu_s * r.nv_s;
        nurbs_desc& d = sl.desc[i];
        d = pd;
        d.nu_s = r.nu_s;
        d.nv_s = r.nv_s;
        d.us_off = (int64_t)cu;
        cu += r.nu_s;
        d.vs_off = (int64_t)cu;
        cu += r.nv_s;
        d.pts_off = sl.res_off[i];
        rseg = emit_run(rseg, sl.tgt_off[i], sl.res_off[i], (int64_t)(3 * npts));
        int64_t dst = sl.res_off[i] + (int64_t)(3 * npts);
        for (int k = 0; k < kGroups; ++k) {
            const int64_t c = grad_count(pd, k);
            gseg = emit_run(gseg, (int64_t)s->gbase[k] + grad_off(pd, k), dst, c);
            dst += c;
        }
    }
    s->pack.run(n, [&](int i) {
        const Req& r = sl.batch[i];
        const nurbs_desc& d = sl.desc[i];
        std::memcpy(huv + d.us_off, r.us, 4 * (size_t)r.nu_s);
        std::memcpy(huv + d.vs_off, r.vs, 4 * (size_t)r.nv_s);
        std::memcpy(htgt + sl.tgt_off[i], r.tgt, 12 * (size_t)r.nu_s * r.nv_s);
    });
    hipError_t e = hipMemcpyAsync(sl.arena, sl.host, o_seg + sizeof(Seg) * nseg, hipMemcpyHostToDevice, sl.st);
    if (e != hipSuccess) return hip_err(s, e, "hipMemcpyAsync(batch inputs)");
    size_t wsq = 0;
    int rc = nurbs_plan_create_in(s->ctx, sl.desc.data(), n, 0, sl.arena + o_tb, end - o_tb, sl.st, &sl.plan,
                                  nullptr, &wsq);
    if (rc) return plan_err(s, s->ctx, rc, "plan");
    if (wsq > o_tb - o_ws) {
        set_err(s, "plan workspace larger than its region");
        return NURBS_EWORKSPACE;
    }
    const float* uv = reinterpret_cast<const float*>(sl.arena);
    const float* tgt = reinterpret_cast<const float*>(sl.arena + o_tgt);
    const Seg* seg = reinterpret_cast<const Seg*>(sl.arena + o_seg);
    float* res = reinterpret_cast<float*>(sl.arena + o_res);
    float* g = reinterpret_cast<float*>(sl.arena + o_g);
    void* wsp = sl.arena + o_ws;
    const size_t wsn = o_tb - o_ws;
    rc = nurbs_plan_fwd(sl.plan, s->ctrl, s->w, s->ku, s->kv, uv, uv, res, wsp, wsn, sl.st);
    if (rc) return plan_err(s, s->ctx, rc, "forward");
    hipLaunchKernelGGL(k_residual, dim3((unsigned)nrs), dim3(256), 0, sl.st, seg, res, tgt, g);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(s, e, "launch residual");
    float* gf = sl.gflat;
    rc = nurbs_plan_bwd(sl.plan, s->ctrl, s->w, s->ku, s->kv, uv, uv, g, gf + s->gbase[0], gf + s->gbase[1],
                        gf + s->gbase[2], gf + s->gbase[3], NURBS_GRAD_ALL, wsp, wsn, sl.st);
    if (rc) return plan_err(s, s->ctx, rc, "backward");
    hipLaunchKernelGGL(k_copy_segs, dim3((unsigned)ngs), dim3(256), 0, sl.st, seg + nrs, gf, res);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(s, e, "launch gradient gather");
    e = hipMemcpyAsync(sl.host + o_res, sl.arena + o_res, 4 * n_res, hipMemcpyDeviceToHost, sl.st);
    if (e != hipSuccess) return hip_err(s, e, "hipMemcpyAsync(results)");
    e = hipEventRecord(sl.ev, sl.st);
    if (e != hipSuccess) return hip_err(s, e, "hipEventRecord");
    sl.res_o = o_res;
    return NURBS_OK;
}

int free_slot(nurbs_server* s) {
    for (size_t k = 0; k < s->slots.size(); ++k)
        if (!s->slots[k].busy) return (int)k;
    return -1;
}

void engine(nurbs_server* s) {
    (void)hipSetDevice(s->device);
    std::vector<int> take;
    for (;;) {
        int k = -1;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_eng.wait(lk, [&] { return (s->stop && s->pending.empty()) || (!s->pending.empty() && free_slot(s) >= 0); });
            if (s->pending.empty()) break;
            k = free_slot(s);
            auto& q = s->pending;
            admit((int)q.size(), [&](int i) { return q[i].surf; }, [&](int i) { return q[i].nbytes; },
                  s->slot_bytes, s->fixed, s->max_req, take);
            Slot& sl = s->slots[k];
            sl.batch.clear();
            for (int i : take) sl.batch.push_back(q[i]);
            // remove the taken requests; the ones passed over before the last
            // taken one go back to the front, in arrival order
            if (!take.empty()) {
                std::vector<Req> keep;
                for (int i = 0, t = 0; i <= take.back(); ++i) {
                    if (take[t] == i) ++t;
                    else keep.push_back(q[i]);
                }
                q.erase(q.begin(), q.begin() + take.back() + 1);
                q.insert(q.begin(), keep.begin(), keep.end());
            }
            sl.busy = true;
        }
        Slot& sl = s->slots[k];
        const double t0 = now_s();
        if (sl.plan) {  // the slot's previous batch has completed
            nurbs_plan_destroy(sl.plan);
            sl.plan = nullptr;
        }
        const int rc = sl.batch.empty() ? NURBS_EWORKSPACE : launch(s, sl);
        // a failed launch may have queued part of its work: let it drain
        // before the slot's buffers are reused
        if (rc) (void)hipStreamSynchronize(sl.st);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            sl.rc = rc;
            s->launched.push_back(k);
            ++s->batches;
            s->eng_busy += now_s() - t0;
        }
        s->cv_fin.notify_one();
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->eng_done = true;
    }
    s->cv_fin.notify_one();
}

void completer(nurbs_server* s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        int k;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_fin.wait(lk, [&] { return !s->launched.empty() || s->eng_done; });
            if (s->launched.empty()) break;
            k = s->launched.front();
            s->launched.pop_front();
        }
        Slot& sl = s->slots[k];
        int rc = sl.rc;
        if (rc == NURBS_OK) {
            const hipError_t e = hipEventSynchronize(sl.ev);
            if (e != hipSuccess) rc = hip_err(s, e, "batch");
        }
        const double t = now_s();
        if (rc == NURBS_OK) {
            const float* res = reinterpret_cast<const float*>(sl.host + sl.res_o);
            s->unpack.run((int)sl.batch.size(), [&](int i) {
                const Req& r = sl.batch[i];
                std::memcpy(r.out, res + sl.res_off[i], 4 * (size_t)out_floats(s->pool[r.surf], r.nu_s, r.nv_s));
            });
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (const Req& r : sl.batch) {
                s->state[r.id] = rc;
                s->lat[r.id] = t - r.t_arr;
            }
            s->completed += (int64_t)sl.batch.size();
            s->fin_busy += now_s() - t;
            while (s->low < (int64_t)s->state.size() && s->state[s->low] != kPendingState) ++s->low;
            sl.busy = false;
        }
        s->cv_done.notify_all();
        s->cv_eng.notify_one();
    }
}

}  // namespace

extern "C" {

int nurbs_server_admit(const int32_t* surf, const size_t* nbytes, int n, size_t capacity, size_t fixed_bytes,
                       int max_requests, int32_t* take, int* n_take) {
    if (n < 0 || max_requests < 1 || (n > 0 && (!surf || !nbytes || !take)) || !n_take) return NURBS_EINVAL;
    std::vector<int> t;
    admit(n, [&](int i) { return (int)surf[i]; }, [&](int i) { return nbytes[i]; }, capacity, fixed_bytes,
          max_requests, t);
    for (size_t i = 0; i < t.size(); ++i) take[i] = t[i];
    *n_take = (int)t.size();
    return NURBS_OK;
}

int nurbs_server_create(int device, const nurbs_desc* pool, int n_surf, const float* ctrl, const float* w,
                        const float* ku, const float* kv, int n_slots, size_t slot_bytes, int max_requests,
                        nurbs_server** out) {
    if (!out) return NURBS_EINVAL;
    *out = nullptr;
    if (!pool || n_surf < 1 || !ctrl || !w || !ku || !kv || n_slots < 1 || n_slots > 16 || max_requests < 1 ||
        max_requests > (1 << 16) || slot_bytes < (1u << 16))
        return NURBS_EINVAL;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return NURBS_EDEVICE;
    nurbs_server* s = new nurbs_server();
    s->device = device;
    s->pool.assign(pool, pool + n_surf);
    s->ctrl = ctrl;
    s->w = w;
    s->ku = ku;
    s->kv = kv;
    s->slot_bytes = slot_bytes;
    s->max_req = max_requests;
    // fixed bytes of a batch: the plan's workspace header and the alignment of its eight regions
    s->fixed = NURBS_PLAN_WS_HEADER + 8 * kAlign;
    int64_t len[kGroups] = {0, 0, 0, 0};
    for (const nurbs_desc& d : s->pool)
        for (int k = 0; k < kGroups; ++k) len[k] = std::max(len[k], grad_off(d, k) + grad_count(d, k));
    for (int k = 0; k < kGroups; ++k) {
        s->gbase[k] = s->gtotal;
        s->gtotal += (size_t)len[k];
    }
    int rc = nurbs_ctx_create(device, &s->ctx);
    if (rc == NURBS_OK) rc = nurbs_ctx_create(device, &s->qctx);
    s->slots.resize(n_slots);
    for (Slot& sl : s->slots) {
        if (rc) break;
        if ((e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess ||
            (e = hipMalloc(&sl.arena, slot_bytes)) != hipSuccess ||
            (e = hipHostMalloc(&sl.host, slot_bytes, hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc(&sl.gflat, 4 * std::max<size_t>(s->gtotal, 1))) != hipSuccess)
            rc = NURBS_EDEVICE;
    }
    if (rc == NURBS_OK) {
        s->eng = std::thread(engine, s);
        s->fin = std::thread(completer, s);
        *out = s;
        return NURBS_OK;
    }
    for (Slot& sl : s->slots) {
        if (sl.gflat) (void)hipFree(sl.gflat);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.arena) (void)hipFree(sl.arena);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    if (s->qctx) nurbs_ctx_destroy(s->qctx);
    if (s->ctx) nurbs_ctx_destroy(s->ctx);
    delete s;
    return rc;
}

int nurbs_server_submit(nurbs_server* s, int surf, const float* us, int nu_s, const float* vs, int nv_s,
                        const float* target, float* out, double t_arrival, int64_t* id) {
    if (!s || !id) return NURBS_EINVAL;
    *id = -1;
    if (surf < 0 || surf >= (int)s->pool.size() || !us || !vs || !target || !out || nu_s < 1 || nv_s < 1 ||
        nu_s > 65535 || nv_s > 65535)
        return NURBS_EINVAL;
    Req r;
    r.surf = surf;
    r.us = us;
    r.vs = vs;
    r.nu_s = nu_s;
    r.nv_s = nv_s;
    r.tgt = target;
    r.out = out;
    r.t_arr = t_arrival >= 0.0 ? t_arrival : now_s();
    const uint64_t key = ((uint64_t)surf << 32) | ((uint64_t)nu_s << 16) | (uint64_t)nv_s;
    {
        std::lock_guard<std::mutex> lk(s->qmu);
        auto it = s->sizes.find(key);
        if (it == s->sizes.end()) {
            // a plan's sizes depend on the shapes only: asked once per shape
            nurbs_desc d = s->pool[surf];
            d.nu_s = nu_s;
            d.nv_s = nv_s;
            d.us_off = d.vs_off = d.pts_off = 0;
            size_t tb = 0, wb = 0;
            const int rc = nurbs_plan_create_in(s->qctx, &d, 1, 0, nullptr, 0, nullptr, nullptr, &tb, &wb);
            if (rc) return rc;
            it = s->sizes.emplace(key, std::array<size_t, 2>{wb, tb}).first;
        }
        r.ws = it->second[0];
        r.tb = it->second[1];
    }
    const size_t npts = (size_t)nu_s * nv_s;
    const size_t nout = (size_t)out_floats(s->pool[surf], nu_s, nv_s);
    // parameters, targets, segment records, result and dL/dS blocks, workspace tiles, tables
    const size_t nseg = (size_t)(residual_segs(nu_s, nv_s) + gather_segs(s->pool[surf]));
    r.nbytes = 4 * ((size_t)nu_s + nv_s) + 12 * npts + nseg * sizeof(Seg) + 2 * 4 * nout +
               (r.ws - NURBS_PLAN_WS_HEADER) + r.tb;
    if (s->fixed + r.nbytes > s->slot_bytes) return NURBS_EWORKSPACE;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return NURBS_EINVAL;
        r.id = (int64_t)s->state.size();
        s->state.push_back(kPendingState);
        s->lat.push_back(0.0);
        s->pending.push_back(r);
    }
    s->cv_eng.notify_one();
    *id = r.id;
    return NURBS_OK;
}

int nurbs_server_wait(nurbs_server* s, int64_t id, double* latency) {
    if (!s) return NURBS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (id < 0 || id >= (int64_t)s->state.size()) return NURBS_EINVAL;
    s->cv_done.wait(lk, [&] { return s->state[id] != kPendingState; });
    if (latency) *latency = s->lat[id];
    return s->state[id];
}

int nurbs_server_stats(nurbs_server* s, int64_t* batches, int64_t* completed, int64_t* finished_below) {
    if (!s) return NURBS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (batches) *batches = s->batches;
    if (completed) *completed = s->completed;
    if (finished_below) *finished_below = s->low;
    return NURBS_OK;
}

int nurbs_server_busy(nurbs_server* s, double* engine_s, double* completion_s) {
    if (!s) return NURBS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (engine_s) *engine_s = s->eng_busy;
    if (completion_s) *completion_s = s->fin_busy;
    return NURBS_OK;
}

const char* nurbs_server_last_error(nurbs_server* s) {
    thread_local std::string copy;
    if (!s) return "";
    std::lock_guard<std::mutex> lk(s->mu);
    copy = s->err;
    return copy.c_str();
}

int nurbs_server_destroy(nurbs_server* s) {
    if (!s) return NURBS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_eng.notify_all();
    if (s->eng.joinable()) s->eng.join();
    if (s->fin.joinable()) s->fin.join();
    for (Slot& sl : s->slots) {
        if (sl.plan) nurbs_plan_destroy(sl.plan);
        (void)hipFree(sl.gflat);
        (void)hipHostFree(sl.host);
        (void)hipFree(sl.arena);
        (void)hipEventDestroy(sl.ev);
        (void)hipStreamDestroy(sl.st);
    }
    nurbs_ctx_destroy(s->qctx);
    nurbs_ctx_destroy(s->ctx);
    delete s;
    return NURBS_OK;
}

}  // extern "C"
