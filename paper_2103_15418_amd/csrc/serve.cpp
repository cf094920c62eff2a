// Serving loop: many image streams of different shapes on one GPU.
//
// Client threads admit streams (bounded by an HBM budget) and submit frames
// with their arrival stamps.  One dispatcher thread owns every library call:
// in arrival order it launches a frame of each stream that is idle (ingest ->
// detect -> extract_flux, asynchronous on that stream's own HIP stream, so
// frames of different streams overlap on the device), polls the streams'
// completion events, and for all streams whose frame finished runs one pooled
// network batch over the episodes that ended there.  A frame is done when its
// inference rows are back on the host; its latency is done - arrival.

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "lpf_internal.h"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct SrvFrame {
    int64_t t;
    const float* cube;
    int on_device;
    int64_t arrival;
};

struct Recorded {
    std::vector<lpf_peak> peaks;
    std::vector<lpf_source> events;
    std::vector<float> mu, L;
    std::vector<int32_t> ids;
};

struct SrvStream {
    int id = -1;
    lpf_config cfg{};
    lpf_ctx* ctx = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t hs = nullptr;
    hipEvent_t ev = nullptr;
    std::deque<SrvFrame> pending;
    bool busy = false;      // a frame is launched and not yet done
    bool launched = false;  // its kernels are enqueued (waiting for the event)
    bool closing = false;
    SrvFrame cur{};
    lpf_frame_result res{};
    Recorded rec;
};

}  // namespace

struct lpf_server {
    const lpf_model* model = nullptr;
    size_t budget = 0, used = 0;
    bool record = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<int, SrvStream*> streams;
    int next_id = 0;
    std::deque<lpf_frame_result> done;
    std::map<std::pair<int, int64_t>, Recorded> recorded;
    int64_t submitted = 0, completed = 0;
    bool stop = false;
    std::thread th;
    std::vector<float> mu_buf, L_buf;
    std::vector<int32_t> src_buf;
};

namespace {

// Launches one frame (dispatcher thread only).
int launch_frame(lpf_server* srv, SrvStream* s) {
    const SrvFrame& f = s->cur;
    s->res = lpf_frame_result{};
    s->res.stream_id = s->id;
    s->res.t = f.t;
    s->res.arrival_ns = f.arrival;
    int rc = lpf_ingest_frame(s->ctx, f.t, f.cube, f.on_device, nullptr);
    if (rc == LPF_OK) {
        if (srv->record) {
            s->rec = Recorded{};
            const int cap = s->cfg.B * s->cfg.peak_cap, ecap = 2 * s->cfg.max_sources;
            s->rec.peaks.resize(cap);
            s->rec.events.resize(ecap);
            int32_t np = 0, ne = 0;
            rc = lpf_detect(s->ctx, s->rec.peaks.data(), cap, &np, s->rec.events.data(), ecap, &ne);
            s->rec.peaks.resize(std::min(np, cap));
            s->rec.events.resize(std::min(ne, ecap));
            if (rc == LPF_EFULL) rc = LPF_OK;
        } else {
            rc = lpf_detect(s->ctx, nullptr, 0, nullptr, nullptr, 0, nullptr);
        }
    }
    if (rc == LPF_OK) rc = lpf_extract_flux(s->ctx);
    if (rc == LPF_OK && hipEventRecord(s->ev, s->hs) != hipSuccess) rc = LPF_EDEVICE;
    s->res.status = rc;
    s->launched = true;
    return rc;
}

// Pooled inference over streams whose frames completed; marks them done.
void finish_frames(lpf_server* srv, std::vector<SrvStream*>& ready) {
    std::vector<lpf_ctx*> ctxs;
    std::vector<SrvStream*> ok;
    size_t cap = 0;
    for (SrvStream* s : ready) {
        if (s->res.status == LPF_OK) {
            ctxs.push_back(s->ctx);
            ok.push_back(s);
            cap += (size_t)s->cfg.max_sources;
        }
    }
    if (!ctxs.empty()) {
        srv->mu_buf.resize(cap * 4);
        srv->L_buf.resize(cap * 10);
        srv->src_buf.resize(cap * 2);
        int32_t n = 0;
        int rc = lpf_infer(ctxs.data(), (int32_t)ctxs.size(), srv->model, nullptr, 0, srv->mu_buf.data(),
                           srv->L_buf.data(), srv->src_buf.data(), (int32_t)cap, &n);
        for (size_t i = 0; i < ok.size(); ++i) {
            SrvStream* s = ok[i];
            lpf_status_t st;
            if (lpf_status(s->ctx, &st) == LPF_OK) {
                s->res.rejected_bands = st.rejected_bands;
                s->res.n_peaks = st.n_peaks;
                s->res.n_new = st.n_new;
                s->res.n_ended = st.n_ended;
            }
            if (rc != LPF_OK) s->res.status = rc;
        }
        if (srv->record && rc == LPF_OK) {
            for (int r = 0; r < n; ++r) {
                SrvStream* s = ok[srv->src_buf[2 * r]];
                s->rec.mu.insert(s->rec.mu.end(), srv->mu_buf.begin() + 4 * r, srv->mu_buf.begin() + 4 * r + 4);
                s->rec.L.insert(s->rec.L.end(), srv->L_buf.begin() + 10 * r, srv->L_buf.begin() + 10 * r + 10);
                s->rec.ids.push_back(srv->src_buf[2 * r + 1]);
            }
        }
    }
    const int64_t tdone = now_ns();
    std::lock_guard<std::mutex> lk(srv->mu);
    for (SrvStream* s : ready) {
        s->res.done_ns = tdone;
        srv->done.push_back(s->res);
        if (srv->record) srv->recorded[{s->id, s->cur.t}] = std::move(s->rec);
        s->busy = false;
        s->launched = false;
        srv->completed++;
    }
    srv->cv_done.notify_all();
}

void dispatcher(lpf_server* srv) {
    for (;;) {
        std::vector<SrvStream*> to_launch, inflight;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            auto has_work = [&] {
                if (srv->stop) return true;
                for (auto& kv : srv->streams) {
                    SrvStream* s = kv.second;
                    if (s->busy || !s->pending.empty()) return true;
                }
                return false;
            };
            srv->cv_work.wait(lk, has_work);
            bool any_busy = false;
            for (auto& kv : srv->streams) any_busy |= kv.second->busy || !kv.second->pending.empty();
            if (srv->stop && !any_busy) return;
            // frames in arrival order across idle streams
            std::vector<SrvStream*> idle;
            for (auto& kv : srv->streams) {
                SrvStream* s = kv.second;
                if (!s->busy && !s->pending.empty()) idle.push_back(s);
                if (s->busy) inflight.push_back(s);
            }
            std::sort(idle.begin(), idle.end(), [](SrvStream* a, SrvStream* b) {
                return a->pending.front().arrival < b->pending.front().arrival;
            });
            for (SrvStream* s : idle) {
                s->cur = s->pending.front();
                s->pending.pop_front();
                s->busy = true;
                to_launch.push_back(s);
            }
        }
        for (SrvStream* s : to_launch) {
            launch_frame(srv, s);
            inflight.push_back(s);
        }
        std::vector<SrvStream*> ready;
        for (SrvStream* s : inflight) {
            if (!s->launched) continue;
            if (s->res.status != LPF_OK) {
                ready.push_back(s);
                continue;
            }
            const hipError_t q = hipEventQuery(s->ev);
            if (q == hipSuccess) ready.push_back(s);
            else if (q != hipErrorNotReady) {
                s->res.status = LPF_EDEVICE;
                ready.push_back(s);
            }
        }
        if (!ready.empty()) finish_frames(srv, ready);
        else if (to_launch.empty()) std::this_thread::yield();
    }
}

void free_stream(SrvStream* s) {
    if (s->ctx) lpf_destroy(s->ctx);
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->hs) (void)hipStreamDestroy(s->hs);
    if (s->ws) (void)hipFree(s->ws);
    delete s;
}

}  // namespace

extern "C" {

int64_t lpf_now_ns(void) { return now_ns(); }

int lpf_server_create(const lpf_model* model, size_t budget, int32_t record, lpf_server** out) {
    if (!model || !out) return LPF_EINVAL;
    lpf_server* srv = new lpf_server();
    srv->model = model;
    srv->budget = budget;
    srv->record = record != 0;
    srv->th = std::thread(dispatcher, srv);
    *out = srv;
    return LPF_OK;
}

void lpf_server_destroy(lpf_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    srv->th.join();
    for (auto& kv : srv->streams) free_stream(kv.second);
    delete srv;
}

int lpf_server_admit(lpf_server* srv, const lpf_config* cfg, int32_t* stream_id) {
    if (!srv || !cfg || !stream_id) return LPF_EINVAL;
    size_t bytes = 0;
    int rc = lpf_workspace_size(cfg, &bytes);
    if (rc != LPF_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->used + bytes > srv->budget) return LPF_ENOMEM;
        srv->used += bytes;  // reserve
    }
    SrvStream* s = new SrvStream();
    s->cfg = *cfg;
    s->cfg.sky_mask = nullptr;
    s->cfg.grid_rows = nullptr;
    s->ws_bytes = bytes;
    hipError_t e = hipMalloc(&s->ws, bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->hs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        rc = lpf_create(cfg, s->ws, bytes, s->hs, &s->ctx);
    } else {
        rc = (e == hipErrorOutOfMemory) ? LPF_ENOMEM : LPF_EDEVICE;
    }
    if (rc != LPF_OK) {
        free_stream(s);
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->used -= bytes;
        return rc;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    s->id = srv->next_id++;
    srv->streams[s->id] = s;
    *stream_id = s->id;
    return LPF_OK;
}

int lpf_server_close(lpf_server* srv, int32_t id) {
    if (!srv) return LPF_EINVAL;
    SrvStream* s = nullptr;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->streams.find(id);
        if (it == srv->streams.end()) return LPF_EINVAL;
        s = it->second;
        s->closing = true;
        srv->cv_done.wait(lk, [&] { return !s->busy && s->pending.empty(); });
        srv->streams.erase(it);
    }
    const size_t bytes = s->ws_bytes;
    free_stream(s);
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->used -= bytes;
    return LPF_OK;
}

int lpf_server_submit(lpf_server* srv, int32_t id, int64_t t, const float* cube, int32_t on_device,
                      int64_t arrival_ns) {
    if (!srv || !cube) return LPF_EINVAL;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->streams.find(id);
        if (it == srv->streams.end() || it->second->closing) return LPF_EINVAL;
        it->second->pending.push_back(SrvFrame{t, cube, on_device, arrival_ns});
        srv->submitted++;
    }
    srv->cv_work.notify_one();
    return LPF_OK;
}

int lpf_server_poll(lpf_server* srv, lpf_frame_result* out, int32_t cap, int32_t* n) {
    if (!srv || !n || (cap > 0 && !out)) return LPF_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    int k = 0;
    while (k < cap && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *n = k;
    return LPF_OK;
}

int lpf_server_drain(lpf_server* srv) {
    if (!srv) return LPF_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->completed >= srv->submitted; });
    return LPF_OK;
}

int lpf_server_fetch(lpf_server* srv, int32_t id, int64_t t, lpf_peak* peaks, int32_t peak_cap, int32_t* n_peaks,
                     lpf_source* events, int32_t ev_cap, int32_t* n_events, float* mu, float* L, int32_t* ids,
                     int32_t inf_cap, int32_t* n_inf) {
    if (!srv) return LPF_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->recorded.find({id, t});
    if (it == srv->recorded.end()) return LPF_EINVAL;
    const Recorded& r = it->second;
    if (n_peaks) *n_peaks = (int32_t)r.peaks.size();
    if (peaks) std::memcpy(peaks, r.peaks.data(), std::min<size_t>(peak_cap, r.peaks.size()) * sizeof(lpf_peak));
    if (n_events) *n_events = (int32_t)r.events.size();
    if (events)
        std::memcpy(events, r.events.data(), std::min<size_t>(ev_cap, r.events.size()) * sizeof(lpf_source));
    const size_t ni = r.ids.size();
    if (n_inf) *n_inf = (int32_t)ni;
    const size_t k = std::min<size_t>(inf_cap, ni);
    if (mu) std::memcpy(mu, r.mu.data(), k * 4 * sizeof(float));
    if (L) std::memcpy(L, r.L.data(), k * 10 * sizeof(float));
    if (ids) std::memcpy(ids, r.ids.data(), k * sizeof(int32_t));
    return LPF_OK;
}

int lpf_server_usage(const lpf_server* srv, size_t* used, size_t* budget, int32_t* n_streams) {
    if (!srv) return LPF_EINVAL;
    lpf_server* s = const_cast<lpf_server*>(srv);
    std::lock_guard<std::mutex> lk(s->mu);
    if (used) *used = s->used;
    if (budget) *budget = s->budget;
    if (n_streams) *n_streams = (int32_t)s->streams.size();
    return LPF_OK;
}

}  // extern "C"
