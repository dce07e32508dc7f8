// Serving loop (include/dcfmm.h, "Serving"): resident scenes, continuous
// batching of viewport renders (Alg. 4) over several HIP streams, and
// admission by device footprint from a fixed arena.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "scene.h"

using namespace dc;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
public:
    explicit Arena(size_t size) : size_(size) {
        if (size) free_[0] = size;
    }
    // Offset of a block of n bytes, or SIZE_MAX.
    size_t alloc(size_t n) {
        n = align_up(std::max<size_t>(n, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t n) {
        n = align_up(std::max<size_t>(n, 1));
        used_ -= n;
        auto next = free_.lower_bound(off);
        size_t start = off, len = n;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + n == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

enum class State { Queued, Running, Done, Fetching };

struct Request {
    dc_scene scene = nullptr;
    dc_viewport vp{};
    State state = State::Queued;
    int status = DC_OK;
    size_t out_off = SIZE_MAX, out_bytes = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    long long batch = -1;
    int batch_size = 0;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    void* stage = nullptr;  // pinned descriptor staging of this slot
    size_t stage_bytes = 0;
    bool busy = false;
    size_t scratch_off = SIZE_MAX, scratch_bytes = 0;
    std::vector<long long> tickets;
};

}  // namespace

struct dc_server_s {
    dc_server_opts opts{};
    int device = 0;
    char* arena_base = nullptr;
    Arena arena{0};
    std::vector<Slot> slots;
    std::vector<dc_scene> scenes;
    std::vector<dc_eval_opts> scene_eval;  // render options of scenes[k]

    std::mutex mu;
    std::condition_variable work_cv;  // worker: new requests, freed memory, stop
    std::condition_variable done_cv;  // clients: a request finished
    std::deque<long long> queue;
    std::unordered_map<long long, Request> reqs;
    long long next_ticket = 1, next_batch = 0;
    long long waiting_head = 0;  // oldest request last deferred for memory
    dc_server_stats stats{};
    bool stop = false;
    std::thread worker;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    size_t image_bytes(const dc_viewport& vp) const {
        return (size_t)vp.W * vp.H * 3 * (opts.out_dtype == DC_OUT_F64 ? 8 : 4);
    }
    bool registered(dc_scene s) const {
        return std::find(scenes.begin(), scenes.end(), s) != scenes.end();
    }
    // Render options of a registered scene (under mu, or after registration,
    // which never changes them).
    const dc_eval_opts& eval_of(dc_scene s) const {
        return scene_eval[std::find(scenes.begin(), scenes.end(), s) - scenes.begin()];
    }

    void run();
    bool poll_completions();
    bool launch_next();
    void finish(Slot& sl, int status);
};

// Mark a slot's batch finished, release its scratch and wake waiters.
void dc_server_s::finish(Slot& sl, int status) {
    const double t = now();
    for (long long id : sl.tickets) {
        Request& r = reqs[id];
        r.state = State::Done;
        r.status = status;
        r.t_done = t;
        stats.completed++;
    }
    sl.tickets.clear();
    arena.release(sl.scratch_off, sl.scratch_bytes);
    sl.scratch_off = SIZE_MAX;
    sl.busy = false;
    stats.bytes_in_use = (long long)arena.used();
    done_cv.notify_all();
}

bool dc_server_s::poll_completions() {
    bool any = false;
    for (Slot& sl : slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        int status = q == hipSuccess ? DC_OK : DC_ERR_HIP;
        if (status == DC_OK && !sl.tickets.empty()) {
            try {
                fmm_check_stall(*reqs[sl.tickets[0]].scene->fmm);
            } catch (const Error& e) {
                status = e.code;
            }
        }
        finish(sl, status);
        any = true;
    }
    return any;
}

// Form and launch one batch on a free slot.  Returns false when nothing was
// launched (no free slot, empty queue, or the oldest request must wait for
// memory).
bool dc_server_s::launch_next() {
    Slot* sl = nullptr;
    for (Slot& s : slots)
        if (!s.busy) {
            sl = &s;
            break;
        }
    if (!sl || queue.empty()) return false;
    const long long head = queue.front();
    dc_scene sc = reqs[head].scene;
    std::vector<long long> pick;
    long long pixels = 0;
    for (long long id : queue) {
        const Request& r = reqs[id];
        if (r.scene != sc) continue;
        const long long px = (long long)r.vp.W * r.vp.H;
        if (!pick.empty() &&
            ((int)pick.size() >= opts.max_batch || pixels + px > opts.max_batch_pixels))
            break;
        pick.push_back(id);
        pixels += px;
    }
    // Largest prefix of the pick whose images and scratch fit the arena.
    RenderPlan pl;
    std::vector<dc_viewport> vps;
    std::vector<size_t> out_off;
    size_t scratch_off = SIZE_MAX;
    const dc_eval_opts ev = eval_of(sc);
    while (!pick.empty()) {
        vps.clear();
        for (long long id : pick) vps.push_back(reqs[id].vp);
        plan_render(*sc->fmm, vps.data(), (int)vps.size(), ev.tile_px, ev.p, pl);
        out_off.clear();
        bool ok = true;
        for (long long id : pick) {
            const size_t off = arena.alloc(reqs[id].out_bytes);
            if (off == SIZE_MAX) {
                ok = false;
                break;
            }
            out_off.push_back(off);
        }
        if (ok) {
            scratch_off = arena.alloc(pl.scratch_bytes);
            ok = scratch_off != SIZE_MAX;
        }
        if (ok) break;
        for (size_t k = 0; k < out_off.size(); ++k) arena.release(out_off[k], reqs[pick[k]].out_bytes);
        pick.pop_back();
    }
    if (pick.empty()) {
        if (waiting_head != head) {
            stats.admission_waits++;
            waiting_head = head;
        }
        return false;
    }
    // pinned staging of the descriptor tables (a free slot's last copy has
    // completed)
    try {
        if (sl->stage_bytes < pl.desc_bytes) {
            if (sl->stage) DC_HIP(hipHostFree(sl->stage));
            sl->stage = nullptr;
            sl->stage_bytes = 0;
            DC_HIP(hipHostMalloc(&sl->stage, pl.desc_bytes, hipHostMallocDefault));
            sl->stage_bytes = pl.desc_bytes;
        }
    } catch (const Error& e) {
        arena.release(scratch_off, pl.scratch_bytes);
        const double t = now();
        for (size_t k = 0; k < pick.size(); ++k) {
            Request& r = reqs[pick[k]];
            r.out_off = out_off[k];  // released by fetch
            r.state = State::Done;
            r.status = e.code;
            r.t_start = r.t_done = t;
            queue.erase(std::find(queue.begin(), queue.end(), pick[k]));
            stats.completed++;
        }
        done_cv.notify_all();
        return true;
    }
    const long long batch = next_batch++;
    const double t = now();
    std::vector<void*> outs;
    for (size_t k = 0; k < pick.size(); ++k) {
        Request& r = reqs[pick[k]];
        r.out_off = out_off[k];
        r.state = State::Running;
        r.t_start = t;
        r.batch = batch;
        r.batch_size = (int)pick.size();
        outs.push_back(arena_base + r.out_off);
        queue.erase(std::find(queue.begin(), queue.end(), pick[k]));
    }
    pl.write_tables(sl->stage, outs.data());
    sl->busy = true;
    sl->tickets = pick;
    sl->scratch_off = scratch_off;
    sl->scratch_bytes = pl.scratch_bytes;
    stats.batches++;
    stats.bytes_in_use = (long long)arena.used();
    stats.bytes_peak = (long long)arena.peak();
    try {
        fmm_launch_render(*sc, pl, ev, opts.out_dtype, arena_base + scratch_off, sl->stage,
                          sl->st);
        DC_HIP(hipEventRecord(sl->done, sl->st));
    } catch (const Error&) {
        // nothing of this batch may still be queued behind a failed launch
        (void)hipStreamSynchronize(sl->st);
        finish(*sl, DC_ERR_HIP);
    }
    long long running = 0;
    for (const Slot& s : slots) running += s.busy ? 1 : 0;
    stats.max_in_flight = std::max(stats.max_in_flight, running);
    return true;
}

void dc_server_s::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progressed = poll_completions();
        try {
            while (launch_next()) progressed = true;
        } catch (const std::exception& e) {
            // Host-side failure while forming the oldest request's batch
            // (requests were validated at submit, so this is resource
            // exhaustion): fail that request, keep serving the others.
            const long long id = queue.front();
            queue.pop_front();
            Request& r = reqs[id];
            const Error* de = dynamic_cast<const Error*>(&e);
            r.status = de ? de->code : DC_ERR_OOM;
            r.state = State::Done;
            r.t_start = r.t_done = now();
            stats.completed++;
            done_cv.notify_all();
            progressed = true;
        }
        bool busy = false;
        for (const Slot& s : slots) busy = busy || s.busy;
        if (stop && !busy && queue.empty()) break;
        if (progressed) continue;
        if (busy) {
            // batches in flight: poll their events at a short interval
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            work_cv.wait(lk);
        }
    }
}

extern "C" {

void dc_default_server_opts(dc_server_opts* o) {
    if (!o) return;
    dc_default_eval_opts(&o->eval);
    o->eval.precision = DC_PREC_F32;
    o->eval.p = 12;
    o->eval.tile_px = 8;
    o->out_dtype = DC_OUT_F32;
    o->n_streams = 4;
    o->max_batch = 64;
    o->max_batch_pixels = 1LL << 26;
    o->hbm_budget = 8LL << 30;
}

int dc_server_create(const dc_server_opts* o, dc_server* out) {
    return guarded([&] {
        DC_REQUIRE(o && out, "null argument");
        *out = nullptr;
        DC_REQUIRE(o->eval.method == DC_METHOD_FMM, "the server renders with the FMM");
        DC_REQUIRE(o->eval.precision == DC_PREC_F64 || o->eval.precision == DC_PREC_F32,
                   "bad precision");
        DC_REQUIRE(o->eval.p >= 1 && o->eval.p <= DC_P_MAX, "bad expansion order");
        DC_REQUIRE(o->eval.tile_px >= 2 && o->eval.tile_px <= 16, "bad tile_px");
        DC_REQUIRE(o->out_dtype == DC_OUT_F32 || o->out_dtype == DC_OUT_F64, "bad out_dtype");
        DC_REQUIRE(o->n_streams >= 1 && o->n_streams <= 16, "n_streams must be in 1..16");
        DC_REQUIRE(o->max_batch >= 1 && o->max_batch_pixels >= 1, "bad batch limits");
        DC_REQUIRE(o->hbm_budget >= (1 << 20), "hbm_budget below 1 MiB");
        auto sv = std::make_unique<dc_server_s>();
        sv->opts = *o;
        DC_HIP(hipGetDevice(&sv->device));
        DC_HIP(hipMalloc(reinterpret_cast<void**>(&sv->arena_base), (size_t)o->hbm_budget));
        sv->arena = Arena((size_t)o->hbm_budget);
        sv->slots.resize(o->n_streams);
        try {
            for (Slot& s : sv->slots) {
                DC_HIP(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
                DC_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
            }
        } catch (...) {
            for (Slot& s : sv->slots) {
                if (s.done) (void)hipEventDestroy(s.done);
                if (s.st) (void)hipStreamDestroy(s.st);
            }
            (void)hipFree(sv->arena_base);
            throw;
        }
        dc_server_s* raw = sv.get();
        sv->worker = std::thread([raw] { raw->run(); });
        *out = sv.release();
    });
}

namespace {

void add_scene(dc_server sv, dc_scene s, const dc_eval_opts& ev) {
    DC_REQUIRE(s->solved, "the scene has no densities (solve or set them first)");
    DC_REQUIRE(ev.method == DC_METHOD_FMM, "the server renders with the FMM");
    DC_REQUIRE(ev.precision == DC_PREC_F64 || ev.precision == DC_PREC_F32, "bad precision");
    DC_REQUIRE(ev.p >= 1 && ev.p <= DC_P_MAX, "bad expansion order");
    DC_REQUIRE(ev.tile_px >= 2 && ev.tile_px <= 16, "bad tile_px");
    DC_REQUIRE(std::isfinite(ev.near_fp64) && ev.near_fp64 >= 0.0, "bad near_fp64");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->registered(s)) {
        const dc_eval_opts& have = sv->eval_of(s);
        DC_REQUIRE(have.p == ev.p && have.precision == ev.precision &&
                       have.tile_px == ev.tile_px && have.near_fp64 == ev.near_fp64,
                   "the scene is registered with this server under other options");
        return;
    }
    const FmmState& f = *s->fmm;
    DC_REQUIRE(s->served.load() == 0 ||
                   (f.up_p == ev.p && f.up_prec == (ev.precision == DC_PREC_F32 ? 4 : 8)),
               "the scene is registered with a server of another order or precision");
    fmm_prepare(*s, ev, nullptr);
    DC_HIP(hipDeviceSynchronize());
    s->served.fetch_add(1);
    sv->scenes.push_back(s);
    sv->scene_eval.push_back(ev);
}

}  // namespace

int dc_server_add_scene(dc_server sv, dc_scene s) {
    return guarded([&] {
        DC_REQUIRE(sv && s, "null argument");
        add_scene(sv, s, sv->opts.eval);
    });
}

int dc_server_add_scene_opts(dc_server sv, dc_scene s, const dc_eval_opts* o) {
    return guarded([&] {
        DC_REQUIRE(sv && s && o, "null argument");
        add_scene(sv, s, *o);
    });
}

int dc_server_submit(dc_server sv, dc_scene s, const dc_viewport* vp, long long* ticket) {
    return guarded([&] {
        DC_REQUIRE(sv && s && vp && ticket, "null argument");
        DC_REQUIRE(vp->W >= 1 && vp->H >= 1 && vp->width > 0 && vp->height > 0 &&
                       std::isfinite(vp->cx) && std::isfinite(vp->cy) &&
                       std::isfinite(vp->width) && std::isfinite(vp->height),
                   "bad viewport");
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            DC_REQUIRE(!sv->stop, "server is shutting down");
            DC_REQUIRE(sv->registered(s), "scene is not registered with this server");
        }
        // The plan of the request alone validates the viewport and gives
        // its smallest footprint (host only; the scene's tree is immutable).
        dc_eval_opts ev;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            ev = sv->eval_of(s);
        }
        RenderPlan pl;
        plan_render(*s->fmm, vp, 1, ev.tile_px, ev.p, pl);
        const size_t img = sv->image_bytes(*vp);
        if (align_up(img) + align_up(pl.scratch_bytes) > (size_t)sv->opts.hbm_budget)
            throw Error(DC_ERR_OOM, "request needs more device memory than hbm_budget");
        std::lock_guard<std::mutex> lk(sv->mu);
        const long long id = sv->next_ticket++;
        Request& r = sv->reqs[id];
        r.scene = s;
        r.vp = *vp;
        r.out_bytes = img;
        r.t_submit = sv->now();
        sv->queue.push_back(id);
        sv->stats.submitted++;
        *ticket = id;
        sv->work_cv.notify_one();
    });
}

int dc_server_wait(dc_server sv, long long ticket, double timeout_s, dc_request_info* info) {
    int rc = DC_OK;
    const int g = guarded([&] {
        DC_REQUIRE(sv, "null server");
        std::unique_lock<std::mutex> lk(sv->mu);
        DC_REQUIRE(sv->reqs.count(ticket), "unknown ticket");
        auto ready = [&] {
            auto it = sv->reqs.find(ticket);
            return it == sv->reqs.end() || it->second.state == State::Done ||
                   it->second.state == State::Fetching;
        };
        if (timeout_s < 0)
            sv->done_cv.wait(lk, ready);
        else if (!sv->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
            rc = DC_ERR_TIMEOUT;
        auto it = sv->reqs.find(ticket);
        DC_REQUIRE(it != sv->reqs.end(), "ticket was fetched by another thread");
        const Request& r = it->second;
        if (info) {
            info->t_submit = r.t_submit;
            info->t_start = r.t_start;
            info->t_done = r.t_done;
            info->batch = r.batch;
            info->batch_size = r.batch_size;
            info->status = r.status;
            info->bytes = (long long)r.out_bytes;
        }
        if (rc == DC_ERR_TIMEOUT) set_last_error("request not finished within the timeout");
    });
    return g != DC_OK ? g : rc;
}

int dc_server_fetch(dc_server sv, long long ticket, void* dst, int dst_is_device) {
    return guarded([&] {
        DC_REQUIRE(sv && dst, "null argument");
        size_t off, bytes;
        int status;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            auto it = sv->reqs.find(ticket);
            DC_REQUIRE(it != sv->reqs.end(), "unknown ticket");
            Request& r = it->second;
            DC_REQUIRE(r.state == State::Done, "request not finished (or being fetched)");
            r.state = State::Fetching;
            off = r.out_off;
            bytes = r.out_bytes;
            status = r.status;
        }
        hipError_t e = hipSuccess;
        if (status == DC_OK) {
            e = hipMemcpy(dst, sv->arena_base + off, bytes,
                          dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
            // A device-to-device hipMemcpy can return before the copy has
            // run.  The region goes back to the arena below, and the next
            // batch (on a stream that does not wait for this one) may write
            // it at once: the copy must be finished first.
            if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (off != SIZE_MAX) sv->arena.release(off, bytes);
            sv->reqs.erase(ticket);
            sv->stats.fetched++;
            sv->stats.bytes_in_use = (long long)sv->arena.used();
            sv->work_cv.notify_one();
        }
        DC_REQUIRE(status == DC_OK, "the request's batch failed");
        if (e != hipSuccess)
            throw Error(DC_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    });
}

int dc_server_get_stats(dc_server sv, dc_server_stats* st) {
    return guarded([&] {
        DC_REQUIRE(sv && st, "null argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        *st = sv->stats;
        st->bytes_peak = (long long)sv->arena.peak();
    });
}

void dc_server_destroy(dc_server sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->work_cv.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    for (Slot& s : sv->slots) {
        if (s.st) (void)hipStreamSynchronize(s.st);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.st) (void)hipStreamDestroy(s.st);
        if (s.stage) (void)hipHostFree(s.stage);
    }
    if (sv->arena_base) (void)hipFree(sv->arena_base);
    for (dc_scene s : sv->scenes) s->served.fetch_sub(1);
    delete sv;
}

}  // extern "C"
