// Request loop over resident meshes (include/fpts_serve.h): FIFO admission
// gated by a device memory pool, same-mesh concatenation into batches, one
// batch per stream, completion times from HIP events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "fpts_internal.hpp"
#include "fpts_serve.h"

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing free ranges.
class Pool {
  public:
    explicit Pool(size_t size) : size_(size) { free_[0] = size; }
    static constexpr size_t npos = (size_t)-1;
    size_t alloc(size_t bytes)
    {
        bytes = up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return npos;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t peak() const { return peak_; }

  private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req {
    int mesh;
    int64_t n;
    const double *pts;
    int32_t *code, *elem;
    double *r, *dist, *out;
    int precision;
    int state = FPTS_REQ_QUEUED;
    double t_submit = 0, t_start = 0, t_done = 0;
    int64_t offset = 0;     // position in its batch
    hipEvent_t ready = nullptr;   // inputs written (recorded on the caller's stream)
};

struct MeshEntry {
    fpts_mesh *m;
    int n_fields;
    const double *field;
};

struct Batch {
    std::vector<int64_t> reqs;
    int stream;
    size_t off = 0, bytes = 0;
    int64_t ntot = 0;
};

}  // namespace

struct fpts_server {
    int device = 0;
    size_t budget = 0;
    int64_t max_batch = 0;
    char *pool_mem = nullptr;
    Pool *pool = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done_ev;
    std::vector<bool> busy;
    hipEvent_t ref_ev = nullptr;
    std::chrono::steady_clock::time_point t0;
    // deques: elements keep their addresses when submit / add_mesh append,
    // so the worker reads them while it launches without holding the lock
    std::deque<MeshEntry> meshes;
    std::deque<Req> reqs;
    std::deque<int64_t> pending;
    std::vector<Batch> running;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::thread worker;
    fpts_server_stats st{};
};

namespace {

double now_us(const fpts_server *s)
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - s->t0)
        .count();
}

// Workspace of one batch: Find and Interpolate in one call when the mesh has
// a field, Find alone otherwise.
size_t batch_ws(const MeshEntry &me, int64_t n)
{
    return me.n_fields > 0 ? fpts_find_eval_workspace_size(me.m, n)
                           : fpts_find_workspace_size(me.m, n);
}

// Device bytes one batch of `nreq` requests with `ntot` points needs:
// workspace plus, when concatenated, staging copies of inputs and outputs.
size_t batch_bytes(const fpts_server *s, int mesh, int64_t ntot, size_t nreq)
{
    const MeshEntry &me = s->meshes[mesh];
    size_t ws = batch_ws(me, ntot);
    if (ws == 0) return (size_t)-1;
    size_t b = up(ws);
    if (nreq > 1) {
        const int D = me.m->D, R = me.m->R;
        b += up(sizeof(double) * D * ntot) + 2 * up(sizeof(int32_t) * ntot) +
             up(sizeof(double) * R * ntot) + up(sizeof(double) * ntot) +
             up(sizeof(double) * std::max(me.n_fields, 1) * ntot);
    }
    return b;
}

// Enqueue one batch on its stream.  Runs without the server lock: the
// requests and the mesh entry are passed by address (taken under the lock;
// deque elements do not move), and nothing here writes shared state.
bool launch(fpts_server *s, const Batch &b, const std::vector<const Req *> &rq,
            const MeshEntry &me)
{
    hipStream_t st = s->streams[b.stream];
    const Req &r0 = *rq[0];
    const int D = me.m->D, R = me.m->R, nf = me.n_fields;
    char *base = s->pool_mem + b.off;
    const int64_t n = b.ntot;
    const double *pts;
    int32_t *code, *elem;
    double *r, *dist, *out;
    char *ws;
    size_t wsb = batch_ws(me, n);
    bool ok = true;
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        if (bytes && hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
            ok = false;
    };
    for (const Req *q : rq)
        if (hipStreamWaitEvent(st, q->ready, 0) != hipSuccess) ok = false;
    if (b.reqs.size() == 1) {
        pts = r0.pts;
        code = r0.code;
        elem = r0.elem;
        r = r0.r;
        dist = r0.dist;
        out = r0.out;
        ws = base;
    } else {
        char *p = base + up(wsb);
        double *pts_b = reinterpret_cast<double *>(p);
        p += up(sizeof(double) * D * n);
        code = reinterpret_cast<int32_t *>(p);
        p += up(sizeof(int32_t) * n);
        elem = reinterpret_cast<int32_t *>(p);
        p += up(sizeof(int32_t) * n);
        r = reinterpret_cast<double *>(p);
        p += up(sizeof(double) * R * n);
        dist = reinterpret_cast<double *>(p);
        p += up(sizeof(double) * n);
        out = reinterpret_cast<double *>(p);
        ws = base;
        for (const Req *qp : rq) {
            const Req &q = *qp;
            for (int d = 0; d < D; ++d)
                cp(pts_b + d * n + q.offset, q.pts + d * q.n, sizeof(double) * q.n);
        }
        pts = pts_b;
    }
    if (!ok) return false;
    if (nf > 0) {
        if (fpts_find_eval(me.m, n, pts, code, elem, r, dist, r0.precision, nf, me.m->N, me.field,
                           out, ws, wsb, st) != FPTS_OK)
            return false;
    } else if (fpts_find(me.m, n, pts, code, elem, r, dist, r0.precision, ws, wsb, st) !=
               FPTS_OK) {
        return false;
    }
    if (b.reqs.size() > 1) {
        for (const Req *qp : rq) {
            const Req &q = *qp;
            cp(q.code, code + q.offset, sizeof(int32_t) * q.n);
            cp(q.elem, elem + q.offset, sizeof(int32_t) * q.n);
            cp(q.dist, dist + q.offset, sizeof(double) * q.n);
            for (int k = 0; k < R; ++k)
                cp(q.r + k * q.n, r + k * n + q.offset, sizeof(double) * q.n);
            for (int f = 0; f < nf; ++f)
                cp(q.out + f * q.n, out + f * n + q.offset, sizeof(double) * q.n);
        }
    }
    return ok && hipEventRecord(s->done_ev[b.stream], st) == hipSuccess;
}

void finish(fpts_server *s, Batch &b, bool failed)
{
    double t = now_us(s);
    if (!failed) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, s->ref_ev, s->done_ev[b.stream]) == hipSuccess)
            t = 1e3 * ms;
    }
    for (int64_t id : b.reqs) {
        Req &q = s->reqs[id];
        q.state = failed ? FPTS_REQ_FAILED : FPTS_REQ_DONE;
        q.t_done = t;
        if (q.ready) {
            (void)hipEventDestroy(q.ready);
            q.ready = nullptr;
        }
        if (failed) s->st.failed++;
        else s->st.completed++;
    }
    s->pool->release(b.off, b.bytes);
    s->busy[b.stream] = false;
}

void worker_loop(fpts_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // completions
        bool changed = false;
        for (size_t i = 0; i < s->running.size();) {
            hipError_t q = hipEventQuery(s->done_ev[s->running[i].stream]);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            finish(s, s->running[i], q != hipSuccess);
            s->running.erase(s->running.begin() + i);
            changed = true;
        }
        if (changed) s->cv_done.notify_all();
        // admission: FIFO head, plus later requests of the same mesh and
        // precision while the batch fits
        while (!s->pending.empty()) {
            int sidx = -1;
            for (size_t k = 0; k < s->busy.size(); ++k)
                if (!s->busy[k]) {
                    sidx = (int)k;
                    break;
                }
            if (sidx < 0) break;
            const Req &h = s->reqs[s->pending.front()];
            Batch b;
            b.stream = sidx;
            b.reqs.push_back(s->pending.front());
            b.ntot = h.n;
            size_t bytes = batch_bytes(s, h.mesh, b.ntot, 1);
            for (size_t k = 1; k < s->pending.size(); ++k) {
                const Req &q = s->reqs[s->pending[k]];
                if (q.mesh != h.mesh || q.precision != h.precision) continue;
                if (b.ntot + q.n > s->max_batch) continue;
                size_t nb = batch_bytes(s, h.mesh, b.ntot + q.n, b.reqs.size() + 1);
                if (nb > s->budget) continue;
                b.reqs.push_back(s->pending[k]);
                b.ntot += q.n;
                bytes = nb;
            }
            size_t off = s->pool->alloc(bytes);
            if (off == Pool::npos && b.reqs.size() > 1) {
                // fall back to the head alone
                b.reqs.resize(1);
                b.ntot = h.n;
                bytes = batch_bytes(s, h.mesh, b.ntot, 1);
                off = s->pool->alloc(bytes);
            }
            if (off == Pool::npos) break;   // wait for memory to free up
            b.off = off;
            b.bytes = bytes;
            int64_t o = 0;
            const double t = now_us(s);
            for (int64_t id : b.reqs) {
                Req &q = s->reqs[id];
                q.offset = o;
                o += q.n;
                q.state = FPTS_REQ_RUNNING;
                q.t_start = t;
            }
            for (int64_t id : b.reqs)
                s->pending.erase(std::find(s->pending.begin(), s->pending.end(), id));
            s->busy[sidx] = true;
            // enqueue without the lock: submissions meanwhile are neither
            // blocked nor delayed (their timestamps are taken before they
            // lock in any case)
            std::vector<const Req *> rq;
            for (int64_t id : b.reqs) rq.push_back(&s->reqs[id]);
            const MeshEntry *me = &s->meshes[s->reqs[b.reqs[0]].mesh];
            lk.unlock();
            const bool launched = launch(s, b, rq, *me);
            if (!launched) {
                (void)hipGetLastError();
                (void)hipStreamSynchronize(s->streams[sidx]);
            }
            lk.lock();
            if (!launched) {
                finish(s, b, true);
                s->cv_done.notify_all();
                continue;
            }
            s->st.batches++;
            s->st.points += b.ntot;
            s->st.max_batch_requests =
                std::max<int64_t>(s->st.max_batch_requests, (int64_t)b.reqs.size());
            s->running.push_back(std::move(b));
            s->st.max_in_flight = std::max<int64_t>(s->st.max_in_flight, s->running.size());
        }
        if (s->stop && s->pending.empty() && s->running.empty()) break;
        if (s->running.empty()) {
            s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
        } else {
            // poll the running batches' events
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

extern "C" {

int fpts_server_create(size_t budget_bytes, int n_streams, int64_t max_batch_points,
                       fpts_server **out)
{
    if (!out || budget_bytes < ((size_t)1 << 20) || n_streams < 1 || n_streams > 16 ||
        max_batch_points < 1)
        return FPTS_EINVAL;
    *out = nullptr;
    fpts_server *s = new (std::nothrow) fpts_server();
    if (!s) return FPTS_ENOMEM;
    s->budget = budget_bytes;
    s->max_batch = std::min<int64_t>(max_batch_points, INT32_MAX - 1);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return FPTS_EDEVICE;
    }
    if (hipMalloc(&s->pool_mem, budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return FPTS_ENOMEM;
    }
    s->pool = new Pool(budget_bytes);
    s->streams.resize(n_streams);
    s->done_ev.resize(n_streams);
    s->busy.assign(n_streams, false);
    bool ok = true;
    for (int k = 0; k < n_streams; ++k)
        ok = ok && hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreate(&s->done_ev[k]) == hipSuccess;
    ok = ok && hipEventCreate(&s->ref_ev) == hipSuccess &&
         hipEventRecord(s->ref_ev, s->streams[0]) == hipSuccess &&
         hipEventSynchronize(s->ref_ev) == hipSuccess;
    s->t0 = std::chrono::steady_clock::now();
    if (!ok) {
        (void)hipGetLastError();
        fpts_server_destroy(s);
        return FPTS_EDEVICE;
    }
    s->st.budget_bytes = budget_bytes;
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return FPTS_OK;
}

int fpts_server_destroy(fpts_server *s)
{
    if (!s) return FPTS_OK;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->worker.join();
    }
    for (auto st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    for (auto e : s->done_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->ref_ev) (void)hipEventDestroy(s->ref_ev);
    (void)hipFree(s->pool_mem);
    delete s->pool;
    delete s;
    return FPTS_OK;
}

int fpts_server_add_mesh(fpts_server *s, fpts_mesh *m, int n_fields, const double *d_field,
                         int *mesh_id)
{
    if (!s || !m || !mesh_id || n_fields < 0 || (n_fields > 0 && !d_field)) return FPTS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    s->meshes.push_back(MeshEntry{m, n_fields, d_field});
    *mesh_id = (int)s->meshes.size() - 1;
    return FPTS_OK;
}

int fpts_server_submit(fpts_server *s, int mesh_id, int64_t n, const double *d_pts,
                       int32_t *d_code, int32_t *d_elem, double *d_r, double *d_dist,
                       double *d_out, int precision, void *stream, int64_t *req_id)
{
    if (!s || !req_id || n < 1 || !d_pts || !d_code || !d_elem || !d_r || !d_dist)
        return FPTS_EINVAL;
    if (precision != FPTS_FP64 && precision != FPTS_MIXED) return FPTS_EINVAL;
    const double t_submit = now_us(s);
    hipEvent_t ready = nullptr;
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ready, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        if (ready) (void)hipEventDestroy(ready);
        return FPTS_EDEVICE;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    int bad = FPTS_OK;
    if (mesh_id < 0 || mesh_id >= (int)s->meshes.size()) bad = FPTS_EINVAL;
    else if (s->meshes[mesh_id].n_fields > 0 && !d_out) bad = FPTS_EINVAL;
    else if (n > s->max_batch) bad = FPTS_EINVAL;
    else if (batch_bytes(s, mesh_id, n, 1) > s->budget) bad = FPTS_ENOMEM;
    if (bad != FPTS_OK) {
        lk.unlock();
        (void)hipEventDestroy(ready);
        return bad;
    }
    Req q;
    q.mesh = mesh_id;
    q.n = n;
    q.pts = d_pts;
    q.code = d_code;
    q.elem = d_elem;
    q.r = d_r;
    q.dist = d_dist;
    q.out = d_out;
    q.precision = precision;
    q.t_submit = t_submit;
    q.ready = ready;
    s->reqs.push_back(q);
    *req_id = (int64_t)s->reqs.size() - 1;
    s->pending.push_back(*req_id);
    s->st.submitted++;
    lk.unlock();
    s->cv_work.notify_all();
    return FPTS_OK;
}

int fpts_server_poll(fpts_server *s, int64_t req_id, int *state, double *t_submit_us,
                     double *t_start_us, double *t_done_us)
{
    if (!s) return FPTS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    if (req_id < 0 || req_id >= (int64_t)s->reqs.size()) return FPTS_EINVAL;
    const Req &q = s->reqs[req_id];
    if (state) *state = q.state;
    if (t_submit_us) *t_submit_us = q.t_submit;
    if (t_start_us) *t_start_us = q.t_start;
    if (t_done_us) *t_done_us = q.t_done;
    return FPTS_OK;
}

int fpts_server_wait(fpts_server *s, int64_t req_id)
{
    if (!s) return FPTS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (req_id < 0 || req_id >= (int64_t)s->reqs.size()) return FPTS_EINVAL;
    s->cv_done.wait(lk, [&] {
        return s->reqs[req_id].state == FPTS_REQ_DONE || s->reqs[req_id].state == FPTS_REQ_FAILED;
    });
    return s->reqs[req_id].state == FPTS_REQ_DONE ? FPTS_OK : FPTS_EDEVICE;
}

int fpts_server_drain(fpts_server *s)
{
    if (!s) return FPTS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->st.completed + s->st.failed == s->st.submitted; });
    return s->st.failed ? FPTS_EDEVICE : FPTS_OK;
}

int fpts_server_stats_get(fpts_server *s, fpts_server_stats *out)
{
    if (!s || !out) return FPTS_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->st;
    out->peak_bytes = s->pool->peak();
    return FPTS_OK;
}

}  // extern "C"
