// Serving runtime of libbfm: requests of different sizes and parameters run as
// they arrive, several at a time on the streams of one device, with admission by
// free stream and by room in a device pool allocated once.  The contract of
// every entry point is in include/bfm.h.
//
// One worker thread per server owns every HIP call of the serving path (launch,
// events, timing).  Completion is signalled by a host function enqueued after
// each request's work on its stream; the host function only records the time
// and wakes the worker (it makes no HIP call).  Client threads only touch the
// queue and the condition variables.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bfm_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
constexpr uint32_t kAllOutputs = BFM_WANT_MAG | BFM_WANT_SIGMA | BFM_WANT_STATUS | BFM_WANT_BETA |
                                 BFM_WANT_RESID | BFM_WANT_MOSUM;

size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over byte offsets [0, size) of the device pool.
class Pool {
public:
    explicit Pool(size_t size)
    {
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t* off)
    {
        if (n == 0) {
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        if (n == 0) return;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;  // offset -> length
};

// Byte layout of a request's outputs in the pool (offsets from the block start).
struct Layout {
    size_t brk = 0, mag = 0, sigma = 0, status = 0, beta = 0, resid = 0, mosum = 0, total = 0;
};

bool layout_of(const bfm_request& r, Layout* L)
{
    if ((r.outputs & ~kAllOutputs) != 0) return false;
    if (r.out_dtype != BFM_OUT_F32 && r.out_dtype != BFM_OUT_F64) return false;
    const size_t P = (size_t)r.P, N = (size_t)r.prm.n_obs, n = (size_t)r.prm.n_hist;
    const size_t p = 2 + 2 * (size_t)r.prm.order;
    const size_t e = r.out_dtype == BFM_OUT_F64 ? 8 : 4;
    size_t at = 0;
    auto take = [&](bool want, size_t bytes, size_t* off) {
        if (!want) return;
        *off = at;
        at += round_up(bytes);
    };
    take(true, 4 * P, &L->brk);
    take(r.outputs & BFM_WANT_MAG, e * P, &L->mag);
    take(r.outputs & BFM_WANT_SIGMA, e * P, &L->sigma);
    take(r.outputs & BFM_WANT_STATUS, P, &L->status);
    take(r.outputs & BFM_WANT_BETA, e * p * P, &L->beta);
    take(r.outputs & BFM_WANT_RESID, e * N * P, &L->resid);
    take(r.outputs & BFM_WANT_MOSUM, e * (N - n) * P, &L->mosum);
    L->total = at;
    return true;
}

struct Req {
    uint64_t id = 0;
    bfm_request r{};
    Layout lay;
    size_t off = 0;
    enum State { QUEUED, RUNNING, DONE } st = QUEUED;
    bool waited_ops = false;  // held at the head of the queue for operator room
    Clock::time_point t_submit, t_admit, t_done;
    bfm_result res{};
};

}  // namespace

struct bfm_server {
    int device = 0;
    size_t pool_bytes = 0;
    char* pool_dev = nullptr;
    Pool pool{0};
    bfm_ctx* ctx = nullptr;
    struct SlotState {
        hipStream_t stream = nullptr;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        Req* req = nullptr;
        bool finished = false;          // set by the host function
        Clock::time_point t_finished;   // when the host function ran
        bfm_server* owner = nullptr;
        int index = 0;
    };
    std::vector<SlotState> slots;
    std::deque<Req*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    uint64_t next_id = 1;
    int64_t running = 0, max_running = 0, completed = 0, operator_waits = 0;
    size_t in_use = 0;
    bool submitted = false;  // the operator budget is fixed from the first request on
};

namespace {

// Runs on a HIP runtime thread once the work enqueued before it on the slot's
// stream has finished.  No HIP call here.
void on_finished(void* p)
{
    auto* st = static_cast<bfm_server::SlotState*>(p);
    bfm_server* s = st->owner;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        st->finished = true;
        st->t_finished = Clock::now();
    }
    s->cv_work.notify_one();
}

double us_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::micro>(b - a).count();
}

void fill_outputs(bfm_server* s, Req* q)
{
    char* base = s->pool_dev + q->off;
    const bfm_request& r = q->r;
    bfm_outputs& o = q->res.out;
    std::memset(&o, 0, sizeof o);
    o.out_dtype = r.out_dtype;
    o.brk = reinterpret_cast<int32_t*>(base + q->lay.brk);
    if (r.outputs & BFM_WANT_MAG) o.mag = base + q->lay.mag;
    if (r.outputs & BFM_WANT_SIGMA) o.sigma = base + q->lay.sigma;
    if (r.outputs & BFM_WANT_STATUS) o.status = reinterpret_cast<uint8_t*>(base + q->lay.status);
    if (r.outputs & BFM_WANT_BETA) o.beta = base + q->lay.beta;
    if (r.outputs & BFM_WANT_RESID) o.resid = base + q->lay.resid;
    if (r.outputs & BFM_WANT_MOSUM) o.mosum = base + q->lay.mosum;
}

void worker_loop(bfm_server* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // Completions signalled by the host functions.  The event timing (a HIP
        // call) is read without the lock the host functions take.
        std::vector<bfm_server::SlotState*> fin;
        for (auto& sl : s->slots)
            if (sl.finished) fin.push_back(&sl);
        std::vector<float> ms(fin.size(), 0.0f);
        if (!fin.empty()) {
            lk.unlock();
            for (size_t i = 0; i < fin.size(); ++i)
                if (fin[i]->req->r.P > 0 && hipEventElapsedTime(&ms[i], fin[i]->ev0, fin[i]->ev1) != hipSuccess)
                    ms[i] = 0.0f;
            lk.lock();
        }
        bool any_done = false;
        for (size_t i = 0; i < fin.size(); ++i) {
            bfm_server::SlotState& sl = *fin[i];
            Req* q = sl.req;
            q->t_done = sl.t_finished;
            q->res.device_us = 1e3 * (double)ms[i];
            q->res.queued_us = us_between(q->t_submit, q->t_admit);
            q->res.latency_us = us_between(q->t_submit, q->t_done);
            q->st = Req::DONE;
            sl.req = nullptr;
            sl.finished = false;
            --s->running;
            ++s->completed;
            any_done = true;
        }
        if (any_done) s->cv_done.notify_all();
        if (s->stop && s->running == 0) break;

        // Admissions, in arrival order: a free stream and room in the pool.
        while (!s->stop && !s->queue.empty()) {
            auto free_slot = std::find_if(s->slots.begin(), s->slots.end(),
                                          [](const bfm_server::SlotState& x) { return !x.req; });
            if (free_slot == s->slots.end()) break;
            Req* q = s->queue.front();
            // HBM footprint: the operators of a parameter set not yet cached
            // must fit next to those that running requests read, and the
            // outputs in the pool.
            if (q->r.P > 0 && !bfm::operator_room(s->ctx, q->r.prm)) {
                if (!q->waited_ops) ++s->operator_waits;
                q->waited_ops = true;
                break;
            }
            if (!s->pool.alloc(q->lay.total, &q->off)) break;
            s->queue.pop_front();
            s->in_use += q->lay.total;
            fill_outputs(s, q);
            q->st = Req::RUNNING;
            q->t_admit = Clock::now();
            free_slot->req = q;
            ++s->running;
            s->max_running = std::max(s->max_running, s->running);
            bfm_server::SlotState* sl = &*free_slot;
            // The launch itself runs without the lock (a first use of a
            // parameter set builds its operators on the host).
            lk.unlock();
            hipStream_t st = sl->stream;
            int rc = BFM_SUCCESS;
            if (q->r.P > 0) {
                (void)hipEventRecord(sl->ev0, st);
                rc = bfm_fit_monitor_typed(s->ctx, &q->r.prm, q->r.Y, q->r.y_dtype, q->r.P, q->r.ld,
                                           q->r.valid, q->r.ldv, &q->res.out, st);
                (void)hipEventRecord(sl->ev1, st);
            }
            q->res.rc = rc;
            hipError_t e = hipLaunchHostFunc(st, on_finished, sl);
            lk.lock();
            if (e != hipSuccess) {  // no completion signal will come: finish it here
                q->res.rc = rc ? rc : BFM_E_HIP;
                sl->finished = true;
                sl->t_finished = Clock::now();
            }
        }
        if (s->stop && s->running == 0) break;
        bool pending = false;
        for (auto& sl : s->slots) pending = pending || sl.finished;
        if (!pending) s->cv_work.wait(lk);
    }
}

int check_request(const bfm_request* r)
{
    if (!r) return BFM_E_INVAL;
    int rc = bfm_check_params(&r->prm, r->P, r->ld);
    if (rc) return rc;
    if (r->y_dtype != BFM_Y_F32 && r->y_dtype != BFM_Y_BF16 && r->y_dtype != BFM_Y_F16) return BFM_E_INVAL;
    if (r->P > 0 && !r->Y) return BFM_E_INVAL;
    if (r->prm.mask_mode == BFM_MASK_EXPLICIT && r->P > 0 && (!r->valid || r->ldv < r->P))
        return r->valid ? BFM_E_LAYOUT : BFM_E_INVAL;
    Layout L;
    if (!layout_of(*r, &L)) return BFM_E_INVAL;
    return BFM_SUCCESS;
}

}  // namespace

extern "C" {

int bfm_request_bytes(const bfm_request* req, size_t* bytes)
{
    if (!req || !bytes) return BFM_E_INVAL;
    Layout L;
    if (req->P < 0 || !layout_of(*req, &L)) return BFM_E_INVAL;
    *bytes = L.total;
    return BFM_SUCCESS;
}

int bfm_server_create(bfm_server** out, int device, int slots, size_t pool_bytes)
{
    if (!out || slots < 1 || slots > 64) return BFM_E_INVAL;
    *out = nullptr;
    bfm_ctx* ctx = nullptr;
    int rc = bfm_create(&ctx, device);
    if (rc) return rc;
    auto s = std::make_unique<bfm_server>();
    s->device = device;
    s->ctx = ctx;
    s->pool_bytes = round_up(pool_bytes);
    s->pool = Pool(s->pool_bytes);
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    hipError_t e = s->pool_bytes ? hipMalloc(&s->pool_dev, s->pool_bytes) : hipSuccess;
    s->slots.resize(slots);
    for (int i = 0; i < slots && e == hipSuccess; ++i) {
        auto& sl = s->slots[i];
        sl.owner = s.get();
        sl.index = i;
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&sl.ev0);
        if (e == hipSuccess) e = hipEventCreate(&sl.ev1);
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        for (auto& sl : s->slots) {
            if (sl.ev0) (void)hipEventDestroy(sl.ev0);
            if (sl.ev1) (void)hipEventDestroy(sl.ev1);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        if (s->pool_dev) (void)hipFree(s->pool_dev);
        bfm_destroy(ctx);
        return e == hipErrorOutOfMemory ? BFM_E_NOMEM : BFM_E_HIP;
    }
    s->worker = std::thread(worker_loop, s.get());
    *out = s.release();
    return BFM_SUCCESS;
}

int bfm_server_submit(bfm_server* s, const bfm_request* req, uint64_t* ticket)
{
    if (!s || !ticket) return BFM_E_INVAL;
    int rc = check_request(req);
    if (rc) return rc;
    auto q = std::make_unique<Req>();
    q->r = *req;
    layout_of(q->r, &q->lay);
    if (q->lay.total > s->pool_bytes) return BFM_E_NOMEM;
    if (bfm::operator_block_bound(q->r.prm) > bfm::operator_budget_of(s->ctx)) return BFM_E_NOMEM;
    q->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return BFM_E_INVAL;
        s->submitted = true;
        q->id = s->next_id++;
        *ticket = q->id;
        s->queue.push_back(q.get());
        s->reqs.emplace(q->id, std::move(q));
    }
    s->cv_work.notify_one();
    return BFM_SUCCESS;
}

int bfm_server_wait(bfm_server* s, uint64_t ticket, int timeout_ms, bfm_result* res)
{
    if (!s || !res) return BFM_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return BFM_E_INVAL;
    Req* q = it->second.get();
    auto done = [&] { return q->st == Req::DONE; };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
        return BFM_E_HIP;
    *res = q->res;
    return BFM_SUCCESS;
}

int bfm_server_release(bfm_server* s, uint64_t ticket)
{
    if (!s) return BFM_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end() || it->second->st != Req::DONE) return BFM_E_INVAL;
        Req* q = it->second.get();
        s->pool.release(q->off, q->lay.total);
        s->in_use -= q->lay.total;
        --s->completed;
        s->reqs.erase(it);
    }
    s->cv_work.notify_one();
    return BFM_SUCCESS;
}

int bfm_server_take(bfm_server* s, uint64_t ticket, const bfm_outputs* dst, void* stream)
{
    if (!s || !dst) return BFM_E_INVAL;
    bfm_outputs src;
    size_t P, N, n, p, e;
    uint32_t want;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end() || it->second->st != Req::DONE) return BFM_E_INVAL;
        const Req* q = it->second.get();
        if (q->res.rc != BFM_SUCCESS || dst->out_dtype != q->r.out_dtype) return BFM_E_INVAL;
        src = q->res.out;
        P = (size_t)q->r.P;
        N = (size_t)q->r.prm.n_obs;
        n = (size_t)q->r.prm.n_hist;
        p = 2 + 2 * (size_t)q->r.prm.order;
        e = q->r.out_dtype == BFM_OUT_F64 ? 8 : 4;
        want = q->r.outputs;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t err = hipSuccess;
    auto copy = [&](void* d, const void* from, bool selected, size_t bytes) {
        if (err == hipSuccess && d && selected && bytes)
            err = hipMemcpyAsync(d, from, bytes, hipMemcpyDeviceToDevice, st);
    };
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    copy(dst->brk, src.brk, true, 4 * P);
    copy(dst->mag, src.mag, want & BFM_WANT_MAG, e * P);
    copy(dst->sigma, src.sigma, want & BFM_WANT_SIGMA, e * P);
    copy(dst->status, src.status, want & BFM_WANT_STATUS, P);
    copy(dst->beta, src.beta, want & BFM_WANT_BETA, e * p * P);
    copy(dst->resid, src.resid, want & BFM_WANT_RESID, e * N * P);
    copy(dst->mosum, src.mosum, want & BFM_WANT_MOSUM, e * (N - n) * P);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (err != hipSuccess) return BFM_E_HIP;
    return bfm_server_release(s, ticket);
}

int bfm_server_get_stats(bfm_server* s, bfm_server_stats* st)
{
    if (!s || !st) return BFM_E_INVAL;
    bfm_cache_stats cs{};
    int rc = bfm_cache_get_stats(s->ctx, &cs);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    st->queued = (int64_t)s->queue.size();
    st->running = s->running;
    st->completed = s->completed;
    st->pool_in_use = (int64_t)s->in_use;
    st->max_running = s->max_running;
    st->operator_entries = cs.entries;
    st->operator_bytes = cs.bytes;
    st->operator_evictions = cs.evictions;
    st->operator_waits = s->operator_waits;
    return BFM_SUCCESS;
}

int bfm_server_operator_budget(bfm_server* s, size_t bytes)
{
    if (!s) return BFM_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->submitted) return BFM_E_INVAL;
    return bfm_operator_budget(s->ctx, bytes);
}

int bfm_server_destroy(bfm_server* s)
{
    if (!s) return BFM_SUCCESS;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Req* q : s->queue) {  // dropped: completes with an error
            q->res.rc = BFM_E_INVAL;
            q->st = Req::DONE;
        }
        s->queue.clear();
    }
    s->cv_work.notify_one();
    if (s->worker.joinable()) s->worker.join();
    s->cv_done.notify_all();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (auto& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.ev0) (void)hipEventDestroy(sl.ev0);
        if (sl.ev1) (void)hipEventDestroy(sl.ev1);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->pool_dev) (void)hipFree(s->pool_dev);
    if (prev >= 0) (void)hipSetDevice(prev);
    bfm_destroy(s->ctx);
    delete s;
    return BFM_SUCCESS;
}

}  // extern "C"
