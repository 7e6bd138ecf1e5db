// Serving loop of the posterior engine (see include/qp.h): families arrive
// over time, are admitted when a slot is free and the device-memory budget
// covers their workspace and outputs, run concurrently on a pool of streams
// (continuous batching: a family admitted while others run overlaps with
// them on the device), and are handed back as host results with their
// submit / admit / done times.  The stage-I work of every family is the same
// computation as qp_posteriors; only the scheduling differs, so a family's
// result does not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "qp.h"
#include "qp_internal.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

enum class St { Queued, Running, Completing, Done, Canceled };

// Device memory of the server: one region of the whole budget, reserved when
// the server is made, from which every admitted family takes one contiguous
// block of the size computed for it at submit (first fit; freed blocks merge
// with their neighbours).  Serving then makes no hipMalloc or hipFree call:
// those synchronise the device and would stall the families in flight.
struct Arena {
    std::mutex mu;
    char* base = nullptr;
    int64_t size = 0;
    std::map<int64_t, int64_t> free_;  // offset -> length of each free range
    int64_t in_use = 0;

    static int64_t round(int64_t b) { return (std::max<int64_t>(b, 1) + 255) & ~int64_t(255); }
    // offset of a block of `bytes`, or -1 when no free range holds it
    int64_t take(int64_t bytes) {
        bytes = round(bytes);
        std::lock_guard<std::mutex> g(mu);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            in_use += bytes;
            return off;
        }
        return -1;
    }
    void give(int64_t off, int64_t bytes) {
        bytes = round(bytes);
        std::lock_guard<std::mutex> g(mu);
        in_use -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
};

// a family's block, handed out piece by piece (256-byte aligned, the same
// rounding the plan's size count uses); pieces go back with the block
struct Bump {
    char* base = nullptr;
    int64_t used = 0, cap = 0;
    static void* alloc(void* ctx, size_t bytes) {
        Bump* b = static_cast<Bump*>(ctx);
        const int64_t need = Arena::round((int64_t)bytes);
        if (b->used + need > b->cap) return nullptr;
        void* p = b->base + b->used;
        b->used += need;
        return p;
    }
    static void release(void*, void*) {}
};

struct Request {
    uint64_t ticket = 0;
    std::vector<uint8_t> codes;   // all sequences concatenated
    std::vector<int64_t> off;     // start of each sequence
    std::vector<int32_t> lens;
    qp_params params{};
    float thresh = 0.f;
    qp_plan* plan = nullptr;      // shaped at submit, materialised at admission
    int64_t bytes = 0;            // device bytes while running
    int64_t cells = 0;
    double t_submit = 0, t_admit = 0, t_done = 0, t_launched = 0, t_device = 0;
    uint8_t* d_codes = nullptr;
    int64_t* d_off = nullptr;
    int64_t block = -1;           // offset of the family's block in the arena
    Bump bump;
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    qp_result* result = nullptr;
    qp_status status = QP_OK;
    std::string error;
    St state = St::Queued;
};

}  // namespace

struct qp_server {
    qp_server_config cfg{};
    int device = 0;
    int64_t wave_budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::vector<Request*> running;
    std::map<uint64_t, Request*> all;
    int64_t bytes_in_use = 0, finished = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    std::thread thr;
    // finished families are downloaded by a second thread, so the scheduler
    // keeps admitting and launching meanwhile
    std::deque<Request*> done_q;
    std::condition_variable cv_comp;
    std::vector<std::thread> comp;
    Arena arena;
};

namespace {

// the family's device work is over (or never started): its plan, event and
// arena block go
void release_device(qp_server* s, Request* r) {
    if (r->plan) qp_plan_destroy(r->plan);  // waits for the plan's last run
    r->plan = nullptr;
    if (r->done_ev) hipEventDestroy(r->done_ev);
    r->d_codes = nullptr;
    r->d_off = nullptr;
    r->done_ev = nullptr;
    if (r->block >= 0) s->arena.give(r->block, r->bytes);
    r->block = -1;
}

// admission (the family's block is taken): upload, enqueue the whole
// pipeline on the stream
qp_status launch(qp_server* s, Request* r) {
    r->bump.base = s->arena.base + r->block;
    r->bump.used = 0;
    r->bump.cap = Arena::round(r->bytes);
    qp::plan_set_allocator(r->plan, qp::DeviceAllocator{&Bump::alloc, &Bump::release, &r->bump});
    qp_status st = qp::plan_materialize(r->plan);
    if (st != QP_OK) return st;
    qp_plan_set_graph(r->plan, 0);
    const int64_t tot = std::max<int64_t>(1, (int64_t)r->codes.size());
    r->d_codes = static_cast<uint8_t*>(Bump::alloc(&r->bump, (size_t)tot));
    r->d_off = static_cast<int64_t*>(Bump::alloc(&r->bump, sizeof(int64_t) * std::max<size_t>(1, r->off.size())));
    hipError_t e = r->d_codes && r->d_off ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return qp::set_error(QP_ENOMEM, "device allocation for an admitted family failed");
    }
    if (!r->codes.empty())
        e = hipMemcpyAsync(r->d_codes, r->codes.data(), r->codes.size(), hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess && !r->off.empty())
        e = hipMemcpyAsync(r->d_off, r->off.data(), sizeof(int64_t) * r->off.size(), hipMemcpyHostToDevice,
                           r->stream);
    if (e != hipSuccess) return qp::set_error(QP_EDEVICE, "host-to-device copy failed");
    st = qp_plan_run(r->plan, r->d_codes, r->d_off, r->stream);
    if (st != QP_OK) return st;
    if (hipEventRecord(r->done_ev, r->stream) != hipSuccess)
        return qp::set_error(QP_EDEVICE, "event record failed");
    return QP_OK;
}

// a family's device work has finished: download its result (its plan holds
// the output bound, so the output always fits)
void complete(qp_server* s, Request* r, qp::Staging* stg) {
    (void)s;
    const qp_status st = qp::plan_download(r->plan, &r->result, stg);
    r->status = st;
    if (st != QP_OK) r->error = qp_last_error();
}

void scheduler(qp_server* s) {
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // admit in arrival order while a slot is free and the reserved
        // device memory holds the next family's block
        while (!s->queue.empty() && (int)s->running.size() < s->cfg.max_slots) {
            Request* r = s->queue.front();
            r->block = s->arena.take(r->bytes);
            if (r->block < 0) break;  // waits for a family to finish
            s->queue.pop_front();
            r->state = St::Running;
            r->t_admit = now_s();
            r->stream = s->streams[s->next_stream++ % s->streams.size()];
            s->running.push_back(r);
            s->bytes_in_use += r->bytes;
            lk.unlock();
            const qp_status st = launch(s, r);
            std::string err = st == QP_OK ? "" : qp_last_error();
            r->t_launched = now_s();
            lk.lock();
            if (st != QP_OK) {
                if (r->stream) hipStreamSynchronize(r->stream);
                release_device(s, r);
                r->status = st;
                r->error = err;
                r->state = St::Done;
                r->t_done = now_s();
                s->bytes_in_use -= r->bytes;
                s->running.erase(std::find(s->running.begin(), s->running.end(), r));
                s->finished++;
                s->cv_done.notify_all();
            }
        }
        // hand families whose device work has finished to the download thread
        bool any_done = false;
        for (Request* r : s->running) {
            if (r->state != St::Running || hipEventQuery(r->done_ev) != hipSuccess) continue;
            r->t_device = now_s();
            r->state = St::Completing;
            s->done_q.push_back(r);
            any_done = true;
        }
        if (any_done) s->cv_comp.notify_all();
        if (s->stop && s->running.empty() && s->queue.empty()) break;
        if (s->running.empty())
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        else
            s->cv_work.wait_for(lk, std::chrono::microseconds(100));
    }
}

// downloads finished families (through its own pinned staging buffer) and
// gives their device memory back to the arena; several run side by side
constexpr int kCompleters = 3;
constexpr size_t kStageHalf = (size_t)32 << 20;

void completer(qp_server* s) {
    hipSetDevice(s->device);
    qp::Staging stg;
    qp::Staging* use = &stg;
    if (hipHostMalloc((void**)&stg.buf, 2 * kStageHalf, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&stg.ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&stg.ev[1], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        use = nullptr;  // direct copies
    } else {
        stg.half = kStageHalf;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_comp.wait(lk, [&] { return !s->done_q.empty() || (s->stop && s->running.empty()); });
        if (s->done_q.empty()) {
            if (s->stop && s->running.empty()) break;
            continue;
        }
        Request* r = s->done_q.front();
        s->done_q.pop_front();
        lk.unlock();
        complete(s, r, use);
        release_device(s, r);
        lk.lock();
        r->t_done = now_s();
        r->state = St::Done;
        s->bytes_in_use -= r->bytes;
        s->running.erase(std::find(s->running.begin(), s->running.end(), r));
        s->finished++;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    lk.unlock();
    if (stg.buf) hipHostFree(stg.buf);
    for (hipEvent_t e : stg.ev)
        if (e) hipEventDestroy(e);
}

}  // namespace

extern "C" {

qp_status qp_server_create(const qp_server_config* cfg, qp_server** out) {
    if (!out) return qp::set_error(QP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return qp::set_error(QP_EINVAL, "config is NULL");
    if (cfg->hbm_budget_bytes <= 0) return qp::set_error(QP_EINVAL, "hbm_budget_bytes must be > 0");
    if (cfg->max_slots < 1 || cfg->max_slots > 64) return qp::set_error(QP_EINVAL, "max_slots must be in 1..64");
    if (cfg->n_streams < 1 || cfg->n_streams > 16) return qp::set_error(QP_EINVAL, "n_streams must be in 1..16");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return qp::set_error(QP_EDEVICE, "no HIP device available");
    }
    qp_server* s = new (std::nothrow) qp_server();
    if (!s) return qp::set_error(QP_ENOMEM, "out of host memory");
    s->cfg = *cfg;
    hipGetDevice(&s->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, s->device) != hipSuccess) {
        delete s;
        return qp::set_error(QP_EDEVICE, "device properties unavailable");
    }
    // each admitted family gets an equal share of four resident waves per
    // SIMD, twice over so that a finishing family's share is taken up by the
    // others (with 4 families in flight a family may fill the device at two
    // waves per SIMD: at the C4 arrival rate that lowered the p99 family
    // latency against three waves per SIMD)
    s->wave_budget = std::max<int64_t>(256, (int64_t)prop.multiProcessorCount * 4 * 4 * 2 / cfg->max_slots);
    for (int q = 0; q < cfg->n_streams; ++q) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) hipStreamDestroy(x);
            delete s;
            return qp::set_error(QP_EDEVICE, "stream creation failed");
        }
        s->streams.push_back(st);
    }
    // the whole budget, reserved once
    if (hipMalloc((void**)&s->arena.base, (size_t)cfg->hbm_budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        for (hipStream_t x : s->streams) hipStreamDestroy(x);
        delete s;
        return qp::set_error(QP_ENOMEM, "the device cannot hold the server's memory budget");
    }
    s->arena.size = cfg->hbm_budget_bytes;
    s->arena.free_[0] = cfg->hbm_budget_bytes & ~int64_t(255);
    s->thr = std::thread(scheduler, s);
    for (int q = 0; q < kCompleters; ++q) s->comp.emplace_back(completer, s);
    *out = s;
    return QP_OK;
}

qp_status qp_server_submit(qp_server* s, const uint8_t* const* seqs, const int32_t* lens, int32_t n,
                           const qp_params* params, float thresh, uint64_t* ticket) {
    if (!s || !ticket) return qp::set_error(QP_EINVAL, "server or ticket is NULL");
    *ticket = 0;
    if (n < 0 || (n > 0 && (!seqs || !lens))) return qp::set_error(QP_EINVAL, "bad family arguments");
    {
        const qp_status pst = qp_params_check(params);  // sets the message
        if (pst != QP_OK) return pst;
    }
    const int alphabet = params->alphabet == 0 ? QP_ALPHA : params->alphabet;
    Request* r = new (std::nothrow) Request();
    if (!r) return qp::set_error(QP_ENOMEM, "out of host memory");
    r->t_submit = now_s();
    int64_t tot = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!seqs[i] || lens[i] < 1) {
            delete r;
            return qp::set_error(QP_EINVAL, "sequence is NULL or empty");
        }
        tot += lens[i];
    }
    r->codes.resize((size_t)tot);
    r->off.resize((size_t)n);
    r->lens.assign(lens, lens + n);
    tot = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t c = 0; c < lens[i]; ++c)
            if (seqs[i][c] >= alphabet) {
                delete r;
                return qp::set_error(QP_EINVAL, "residue code out of range");
            }
        std::memcpy(r->codes.data() + tot, seqs[i], (size_t)lens[i]);
        r->off[i] = tot;
        tot += lens[i];
    }
    r->params = *params;
    r->thresh = thresh;
    for (int32_t i = 0; i + 1 < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) r->cells += (int64_t)lens[i] * lens[j];
    if (n >= 2) {
        // The plan holds the guaranteed output bound at the requested
        // threshold when that fits the budget; otherwise the smallest larger
        // threshold whose bound fits (the memory-budgeted sparsity of the
        // method).  Either way no run can overflow its sparse output.
        const int64_t extra = tot + 8 * (int64_t)n + 1024;  // the family's inputs on the device
        auto shape = [&](float t, int64_t cap, int64_t* bytes) -> qp_status {
            if (r->plan) qp_plan_destroy(r->plan);
            r->plan = nullptr;
            qp_status st = qp::plan_shape(r->lens.data(), n, nullptr, nullptr, 0, params, t, cap, s->wave_budget,
                                          &r->plan);
            if (st != QP_OK) return st;
            qp::plan_set_single_stream(r->plan, true);  // the classes of a family run one after another
            *bytes = qp::plan_bytes(r->plan) + extra;
            return QP_OK;
        };
        int64_t bytes = 0;
        qp_status st = shape(thresh, -1, &bytes);
        if (st == QP_OK && bytes > s->cfg.hbm_budget_bytes) {
            // the same plan with a one-entry output: what the budget must hold
            // besides the sparse output (16 bytes per entry: pool and result)
            int64_t fixed = 0;
            st = shape(thresh, 1, &fixed);
            float t2 = thresh;
            if (st == QP_OK) {
                const int64_t room = (s->cfg.hbm_budget_bytes - fixed) / 16;
                st = room > 0 ? qp_threshold_for_budget(r->lens.data(), n, nullptr, nullptr, 0, room, &t2)
                              : qp::set_error(QP_ENOMEM, "the budget does not hold the family's workspace");
            }
            if (st == QP_OK) st = shape(std::max(thresh, t2), -1, &bytes);
            if (st == QP_OK) r->thresh = std::max(thresh, t2);
        }
        if (st == QP_OK && bytes > s->cfg.hbm_budget_bytes) {
            char msg[160];
            std::snprintf(msg, sizeof(msg), "family needs %lld device bytes, more than the whole budget",
                          (long long)bytes);
            st = qp::set_error(QP_ENOMEM, msg);
        }
        if (st != QP_OK) {
            if (r->plan) qp_plan_destroy(r->plan);
            delete r;
            return st == QP_ENOSPC ? qp::set_error(QP_ENOMEM, "no threshold fits the family in the budget") : st;
        }
        r->bytes = bytes;
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) {
        if (r->plan) qp_plan_destroy(r->plan);
        delete r;
        return qp::set_error(QP_ECANCELED, "server is shutting down");
    }
    r->ticket = s->next_ticket++;
    s->all[r->ticket] = r;
    if (n < 2) {
        // nothing to compute: an immediately finished, empty result
        r->result = qp::result_alloc(n, 0, 0, 0);
        r->state = St::Done;
        r->t_admit = r->t_done = now_s();
        s->finished++;
        s->cv_done.notify_all();
    } else {
        s->queue.push_back(r);
        s->cv_work.notify_all();
    }
    *ticket = r->ticket;
    return QP_OK;
}

qp_status qp_server_wait(qp_server* s, uint64_t ticket, int32_t timeout_ms, qp_result** out,
                         qp_request_times* times) {
    if (out) *out = nullptr;
    if (!s || !out) return qp::set_error(QP_EINVAL, "server or out is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return qp::set_error(QP_EINVAL, "unknown ticket");
    Request* r = it->second;
    auto ready = [&] { return r->state == St::Done || r->state == St::Canceled; };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        return qp::set_error(timeout_ms == 0 ? QP_EBUSY : QP_ETIMEDOUT, "result not ready");
    s->all.erase(it);
    if (times) {
        times->submit_s = r->t_submit;
        times->admit_s = r->t_admit;
        times->done_s = r->t_done;
        times->cells = r->cells;
        times->launched_s = r->t_launched;
        times->device_s = r->t_device;
    }
    qp_status st = r->status;
    if (r->state == St::Canceled) st = QP_ECANCELED;
    if (st == QP_OK) {
        *out = r->result;
        r->result = nullptr;
    } else {
        qp::set_error(st, r->error.empty() ? "request failed" : r->error.c_str());
    }
    if (r->result) qp_result_free(r->result);
    delete r;
    return st;
}

qp_status qp_server_cancel(qp_server* s, uint64_t ticket) {
    if (!s) return qp::set_error(QP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return qp::set_error(QP_EINVAL, "unknown ticket");
    Request* r = it->second;
    if (r->state != St::Queued) return qp::set_error(QP_EBUSY, "request already admitted");
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
    if (r->plan) qp_plan_destroy(r->plan);
    r->plan = nullptr;
    r->state = St::Canceled;
    r->t_done = now_s();
    s->cv_done.notify_all();
    return QP_OK;
}

qp_status qp_server_stats(qp_server* s, int64_t* queued, int64_t* in_flight, int64_t* finished,
                          int64_t* bytes_in_use) {
    if (!s) return qp::set_error(QP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    if (queued) *queued = (int64_t)s->queue.size();
    if (in_flight) *in_flight = (int64_t)s->running.size();
    if (finished) *finished = s->finished;
    if (bytes_in_use) *bytes_in_use = s->bytes_in_use;
    return QP_OK;
}

qp_status qp_server_destroy(qp_server* s) {
    if (!s) return QP_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        // pending requests are cancelled; running ones finish
        for (Request* r : s->queue) {
            if (r->plan) qp_plan_destroy(r->plan);
            r->plan = nullptr;
            r->state = St::Canceled;
        }
        s->queue.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    if (s->thr.joinable()) s->thr.join();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->cv_comp.notify_all();
    }
    for (std::thread& t : s->comp)
        if (t.joinable()) t.join();
    for (auto& kv : s->all) {
        if (kv.second->result) qp_result_free(kv.second->result);
        release_device(s, kv.second);
        delete kv.second;
    }
    for (hipStream_t st : s->streams) hipStreamSynchronize(st);
    hipFree(s->arena.base);
    for (hipStream_t st : s->streams) hipStreamDestroy(st);
    delete s;
    return QP_OK;
}

}  // extern "C"
