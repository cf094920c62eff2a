// Serving loop: many image streams of different shapes on one GPU (Sec. 3.5:
// every stream must keep up with its 1 s cadence).
//
// Client threads admit streams (bounded by an HBM budget; a stream that does
// not fit can wait in a queue until a closed stream frees its share) and
// submit frames with their arrival stamps.  One dispatcher thread owns every
// library call.  Each round it takes the next frame of every idle active
// stream that has one and runs the three per-step stages for all of them as
// batch calls (grouped launches over the streams' contexts, all on the
// server's one HIP stream), then one pooled network ticket over the episodes
// that ended in those streams.  Up to four rounds are in flight; a round is
// done when its ticket's results are on the host, and each of its frames'
// latency is that moment minus the frame's arrival.

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

namespace lpf {
int ticket_state(lpf_model* m, int64_t ticket);
int read_last_lists(lpf_ctx* c, std::vector<lpf_peak>* peaks, std::vector<lpf_source>* events);
}  // namespace lpf

namespace {

using namespace lpf;

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

enum StreamState { kWaiting = 0, kActive = 1 };

struct SrvStream {
    int id = -1;
    int state = kWaiting;
    lpf_config cfg{};
    std::vector<uint8_t> mask;     // copies of the host arrays the config points to
    std::vector<int32_t> rows;
    lpf_ctx* ctx = nullptr;
    void* ws = nullptr;            // workspace: the caller's, or the server's own
    bool own_ws = false;
    size_t ws_bytes = 0;           // what the configuration needs (the budget's unit)
    size_t ws_cap = 0;             // size of an own workspace (a reused one may be larger)
    DevStatus* h_status = nullptr; // pinned copy of the device counters of its current frame
    std::deque<SrvFrame> pending;
    bool busy = false;             // a frame is in a round that is not done
    bool closing = false;
    SrvFrame cur{};
    lpf_frame_result res{};
    Recorded rec;
};

struct Round {
    std::vector<SrvStream*> streams;
    int64_t ticket = -1;
    int status = LPF_OK;
};

}  // namespace

// A closed stream's own workspace and pinned status block, kept for a later
// admission: freeing them would synchronise the whole device mid-serving.
struct PooledWs {
    void* ws;
    size_t cap;
    DevStatus* h_status;
};

struct lpf_server {
    const lpf_model* model = nullptr;
    size_t budget = 0, used = 0;
    std::vector<PooledWs> pool;   // under mu; freed at destroy, or when an admission needs the memory
    size_t pooled = 0;
    bool record = false;
    hipStream_t hs = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<int, SrvStream*> streams;
    std::deque<SrvStream*> waiting;   // admission order
    int next_id = 0;
    std::deque<lpf_frame_result> done;
    std::map<std::pair<int, int64_t>, Recorded> recorded;
    int64_t submitted = 0, completed = 0;
    bool stop = false;
    std::thread th;
    std::deque<Round> rounds;         // in flight, oldest first
    std::vector<float> mu_buf, L_buf;
    std::vector<int32_t> src_buf;
};

namespace {

constexpr int kMaxRounds = kInflight;

// Creates the stream's context on the server's HIP stream (and its own
// workspace if the caller gave none: the smallest pooled one that is large
// enough, else a new one).  Called without the server lock.
int activate(lpf_server* srv, SrvStream* s) {
    lpf_config cfg = s->cfg;
    cfg.sky_mask = s->mask.empty() ? nullptr : s->mask.data();
    cfg.grid_rows = s->rows.empty() ? nullptr : s->rows.data();
    cfg.pipeline_ingest = 0;
    if (!s->ws) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            int best = -1;
            for (int i = 0; i < (int)srv->pool.size(); ++i)
                if (srv->pool[i].cap >= s->ws_bytes && (best < 0 || srv->pool[i].cap < srv->pool[best].cap)) best = i;
            if (best >= 0) {
                s->ws = srv->pool[best].ws;
                s->ws_cap = srv->pool[best].cap;
                s->h_status = srv->pool[best].h_status;
                srv->pooled -= s->ws_cap;
                srv->pool.erase(srv->pool.begin() + best);
            }
        }
        if (!s->ws) {
            if (hipMalloc(&s->ws, s->ws_bytes) != hipSuccess) {
                s->ws = nullptr;
                return LPF_ENOMEM;
            }
            s->ws_cap = s->ws_bytes;
        }
        s->own_ws = true;
    }
    if (!s->h_status &&
        hipHostMalloc(reinterpret_cast<void**>(&s->h_status), sizeof(DevStatus), hipHostMallocDefault) != hipSuccess)
        return LPF_EDEVICE;
    return lpf_create(&cfg, s->ws, s->ws_bytes, srv->hs, &s->ctx);
}

// Ends a stream: its context, then its own workspace and status block back
// to the pool (pool = false: freed, at server destruction).
void free_stream(lpf_server* srv, SrvStream* s, bool pool = true) {
    if (s->ctx) lpf_destroy(s->ctx);   // waits for the stream's work on the server's HIP stream
    if (pool && s->own_ws && s->ws) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->pool.push_back(PooledWs{s->ws, s->ws_cap, s->h_status});
        srv->pooled += s->ws_cap;
    } else {
        if (s->h_status) (void)hipHostFree(s->h_status);
        if (s->own_ws && s->ws) (void)hipFree(s->ws);
    }
    delete s;
}

// Frees pooled workspaces, largest first, until `need` more bytes of the
// server's own allocations fit the budget (caller holds mu).
void trim_pool(lpf_server* srv, size_t need) {
    while (!srv->pool.empty() && srv->used + srv->pooled + need > srv->budget) {
        auto it = std::max_element(srv->pool.begin(), srv->pool.end(),
                                   [](const PooledWs& x, const PooledWs& y) { return x.cap < y.cap; });
        (void)hipHostFree(it->h_status);
        (void)hipFree(it->ws);
        srv->pooled -= it->cap;
        srv->pool.erase(it);
    }
}

// Launches one round over the given streams (dispatcher thread).
void launch_round(lpf_server* srv, std::vector<SrvStream*>& R) {
    Round rd;
    rd.streams = R;
    const int n = (int)R.size();
    std::vector<lpf_ctx*> cs(n);
    std::vector<int64_t> ts(n);
    std::vector<const float*> cubes(n);
    for (int i = 0; i < n; ++i) {
        SrvStream* s = R[i];
        cs[i] = s->ctx;
        ts[i] = s->cur.t;
        cubes[i] = s->cur.cube;
        s->res = lpf_frame_result{};
        s->res.stream_id = s->id;
        s->res.t = s->cur.t;
        s->res.arrival_ns = s->cur.arrival;
        if (srv->record) s->rec = Recorded{};
    }
    int rc = LPF_OK;
    // device and host cubes go through separate ingest calls
    for (int dev = 1; dev >= 0 && rc == LPF_OK; --dev) {
        std::vector<lpf_ctx*> c1;
        std::vector<int64_t> t1;
        std::vector<const float*> q1;
        for (int i = 0; i < n; ++i)
            if ((R[i]->cur.on_device != 0) == (dev != 0)) {
                c1.push_back(cs[i]);
                t1.push_back(ts[i]);
                q1.push_back(cubes[i]);
            }
        if (!c1.empty()) rc = lpf_ingest_batch(c1.data(), t1.data(), q1.data(), dev, (int32_t)c1.size());
    }
    if (rc == LPF_OK) rc = lpf_detect_batch(cs.data(), n);
    if (rc == LPF_OK) rc = lpf_extract_flux_batch(cs.data(), n);
    if (rc == LPF_OK) {
        for (int i = 0; i < n && rc == LPF_OK; ++i)
            if (hipMemcpyAsync(R[i]->h_status, cs[i]->buf.status, sizeof(DevStatus), hipMemcpyDeviceToHost, srv->hs) !=
                hipSuccess)
                rc = LPF_EDEVICE;
    }
    if (rc == LPF_OK && srv->record) {
        for (int i = 0; i < n && rc == LPF_OK; ++i) rc = read_last_lists(cs[i], &R[i]->rec.peaks, &R[i]->rec.events);
    }
    if (rc == LPF_OK) rc = lpf_infer_async(cs.data(), n, const_cast<lpf_model*>(srv->model), &rd.ticket);
    rd.status = rc;
    srv->rounds.push_back(std::move(rd));
}

// Completes the oldest round if its results are in (or wait = true).
// Returns true if a round was completed.
bool finish_round(lpf_server* srv, bool wait) {
    if (srv->rounds.empty()) return false;
    Round& rd = srv->rounds.front();
    lpf_model* m = const_cast<lpf_model*>(srv->model);
    int rc = rd.status;
    int32_t n = 0;
    if (rc == LPF_OK) {
        if (!wait) {
            const int st = ticket_state(m, rd.ticket);
            if (st == 0) return false;
            if (st < 0) rc = LPF_EDEVICE;
        }
        size_t cap = 0;
        for (SrvStream* s : rd.streams) cap += (size_t)s->cfg.max_sources;
        srv->mu_buf.resize(cap * 4);
        srv->L_buf.resize(cap * 10);
        srv->src_buf.resize(cap * 2);
        const int crc = lpf_infer_collect(m, rd.ticket, srv->mu_buf.data(), srv->L_buf.data(), srv->src_buf.data(),
                                          (int32_t)cap, &n);
        if (rc == LPF_OK) rc = crc;
    } else if (rd.ticket >= 0) {
        (void)lpf_infer_collect(m, rd.ticket, nullptr, nullptr, nullptr, 0, &n);
        n = 0;
    }
    if (rc != LPF_OK) {   // the stream's own stream may still run this round's kernels
        (void)hipStreamSynchronize(srv->hs);
    }
    for (size_t i = 0; i < rd.streams.size(); ++i) {
        SrvStream* s = rd.streams[i];
        s->res.status = rc;
        if (rc == LPF_OK) {
            const DevStatus& st = *s->h_status;
            s->res.rejected_bands = st.rejected;
            s->res.n_peaks = st.n_peaks;
            s->res.n_new = st.n_new;
            s->res.n_ended = st.n_ended;
        }
    }
    if (srv->record && rc == LPF_OK) {
        for (int r = 0; r < n; ++r) {
            SrvStream* s = rd.streams[srv->src_buf[2 * r]];
            s->rec.mu.insert(s->rec.mu.end(), srv->mu_buf.begin() + 4 * r, srv->mu_buf.begin() + 4 * r + 4);
            s->rec.L.insert(s->rec.L.end(), srv->L_buf.begin() + 10 * r, srv->L_buf.begin() + 10 * r + 10);
            s->rec.ids.push_back(srv->src_buf[2 * r + 1]);
        }
    }
    const int64_t tdone = now_ns();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (SrvStream* s : rd.streams) {
            s->res.done_ns = tdone;
            srv->done.push_back(s->res);
            if (srv->record) srv->recorded[{s->id, s->cur.t}] = std::move(s->rec);
            s->busy = false;
            srv->completed++;
        }
    }
    srv->rounds.pop_front();
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
    return true;
}

void dispatcher(lpf_server* srv) {
    for (;;) {
        std::vector<SrvStream*> R;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            auto ready = [&] {
                for (auto& kv : srv->streams) {
                    SrvStream* s = kv.second;
                    if (s->state == kActive && !s->busy && !s->pending.empty()) return true;
                }
                return false;
            };
            if (srv->rounds.empty()) {
                srv->cv_work.wait(lk, [&] { return srv->stop || ready(); });
                if (srv->stop && !ready()) return;
            }
            if ((int)srv->rounds.size() < kMaxRounds) {
                // the next frame of every idle active stream, in arrival order
                for (auto& kv : srv->streams) {
                    SrvStream* s = kv.second;
                    if (s->state == kActive && !s->busy && !s->pending.empty()) R.push_back(s);
                }
                std::sort(R.begin(), R.end(), [](SrvStream* a, SrvStream* b) {
                    return a->pending.front().arrival < b->pending.front().arrival;
                });
                for (SrvStream* s : R) {
                    s->cur = s->pending.front();
                    s->pending.pop_front();
                    s->busy = true;
                }
            }
        }
        // a frame out of time order fails alone instead of failing its round
        std::vector<SrvStream*> ok;
        for (SrvStream* s : R) {
            if (s->ctx->n_frames > 0 && s->cur.t <= s->ctx->t_last) {
                lpf_frame_result r{};
                r.stream_id = s->id;
                r.t = s->cur.t;
                r.arrival_ns = s->cur.arrival;
                r.done_ns = now_ns();
                r.status = LPF_EORDER;
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->done.push_back(r);
                srv->completed++;
                s->busy = false;
                srv->cv_done.notify_all();
            } else {
                ok.push_back(s);
            }
        }
        R.swap(ok);
        if (!R.empty()) launch_round(srv, R);
        const bool full = (int)srv->rounds.size() >= kMaxRounds;
        if (!finish_round(srv, full) && R.empty()) std::this_thread::yield();
        while (finish_round(srv, false)) {
        }
    }
}

// Moves waiting streams that now fit the budget to the active set, in
// admission order (caller holds no lock).
void admit_waiting(lpf_server* srv) {
    for (;;) {
        SrvStream* s = nullptr;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (srv->waiting.empty()) return;
            SrvStream* w = srv->waiting.front();
            if (srv->used + w->ws_bytes > srv->budget) return;
            srv->waiting.pop_front();
            if (!w->ws) trim_pool(srv, w->ws_bytes);
            srv->used += w->ws_bytes;
            s = w;
        }
        const int rc = activate(srv, s);
        std::lock_guard<std::mutex> lk(srv->mu);
        if (rc == LPF_OK) {
            s->state = kActive;
        } else {
            // the frames it holds are reported failed
            srv->used -= s->ws_bytes;
            while (!s->pending.empty()) {
                lpf_frame_result r{};
                r.stream_id = s->id;
                r.t = s->pending.front().t;
                r.arrival_ns = s->pending.front().arrival;
                r.done_ns = now_ns();
                r.status = rc;
                srv->done.push_back(r);
                srv->completed++;
                s->pending.pop_front();
            }
            s->state = -1;
        }
        srv->cv_work.notify_all();
        srv->cv_done.notify_all();
    }
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
    if (hipStreamCreateWithFlags(&srv->hs, hipStreamNonBlocking) != hipSuccess) {   // default priority
        delete srv;
        return LPF_EDEVICE;
    }
    srv->th = std::thread(dispatcher, srv);
    *out = srv;
    return LPF_OK;
}

void lpf_server_destroy(lpf_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        // frames of streams that never became active are dropped
        for (SrvStream* s : srv->waiting) s->pending.clear();
    }
    srv->cv_work.notify_all();
    srv->th.join();
    while (finish_round(srv, true)) {
    }
    (void)hipStreamSynchronize(srv->hs);
    for (auto& kv : srv->streams) free_stream(srv, kv.second, false);
    for (const PooledWs& p : srv->pool) {
        (void)hipHostFree(p.h_status);
        (void)hipFree(p.ws);
    }
    (void)hipStreamDestroy(srv->hs);
    delete srv;
}

int lpf_server_admit(lpf_server* srv, const lpf_config* cfg, void* ws, size_t ws_bytes, int32_t queue,
                     int32_t* stream_id, int32_t* active) {
    if (!srv || !cfg || !stream_id) return LPF_EINVAL;
    size_t bytes = 0;
    int rc = lpf_workspace_size(cfg, &bytes);
    if (rc != LPF_OK) return rc;
    if (ws && ws_bytes < bytes) return LPF_ENOMEM;
    SrvStream* s = new SrvStream();
    s->cfg = *cfg;
    s->cfg.sky_mask = nullptr;
    s->cfg.grid_rows = nullptr;
    if (cfg->sky_mask) s->mask.assign(cfg->sky_mask, cfg->sky_mask + (size_t)cfg->H * cfg->W);
    if (cfg->grid_rows) s->rows.assign(cfg->grid_rows, cfg->grid_rows + cfg->B);
    s->ws = ws;
    s->ws_bytes = bytes;
    bool fits;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        fits = srv->waiting.empty() && srv->used + bytes <= srv->budget;
        if (!fits && !queue) {
            delete s;
            return LPF_ENOMEM;
        }
        s->id = srv->next_id++;
        srv->streams[s->id] = s;
        if (fits && !ws) trim_pool(srv, bytes);   // the pool gives way to admitted streams
        if (fits) srv->used += bytes;   // reserve
        else srv->waiting.push_back(s);
    }
    if (fits) {
        rc = activate(srv, s);
        if (rc != LPF_OK) {
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->streams.erase(s->id);
                srv->used -= bytes;
            }
            free_stream(srv, s);   // takes the lock itself
            return rc;
        }
        std::lock_guard<std::mutex> lk(srv->mu);
        s->state = kActive;
    }
    *stream_id = s->id;
    if (active) *active = fits ? 1 : 0;
    return LPF_OK;
}

int lpf_server_close(lpf_server* srv, int32_t id) {
    if (!srv) return LPF_EINVAL;
    SrvStream* s = nullptr;
    bool was_active = false;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->streams.find(id);
        if (it == srv->streams.end()) return LPF_EINVAL;
        s = it->second;
        s->closing = true;
        if (s->state == kWaiting) {
            // never activated: its frames are dropped unprocessed
            srv->waiting.erase(std::find(srv->waiting.begin(), srv->waiting.end(), s));
            srv->completed += (int64_t)s->pending.size();
            s->pending.clear();
        } else {
            srv->cv_done.wait(lk, [&] { return !s->busy && s->pending.empty(); });
        }
        was_active = s->state == kActive;
        srv->streams.erase(it);
        if (was_active) srv->used -= s->ws_bytes;
    }
    free_stream(srv, s);
    srv->cv_done.notify_all();
    admit_waiting(srv);
    return LPF_OK;
}

int lpf_server_submit(lpf_server* srv, int32_t id, int64_t t, const float* cube, int32_t on_device,
                      int64_t arrival_ns) {
    if (!srv || !cube) return LPF_EINVAL;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->streams.find(id);
        if (it == srv->streams.end() || it->second->closing || it->second->state < 0) return LPF_EINVAL;
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
    srv->cv_done.wait(lk, [&] {
        if (srv->completed >= srv->submitted) return true;
        // frames held by waiting streams cannot finish until a stream closes
        int64_t held = 0;
        for (SrvStream* s : srv->waiting) held += (int64_t)s->pending.size();
        return held > 0 && srv->completed + held >= srv->submitted;
    });
    for (SrvStream* s : srv->waiting)
        if (!s->pending.empty()) return LPF_ESTATE;
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
    if (n_streams) *n_streams = (int32_t)(s->streams.size() - s->waiting.size());
    return LPF_OK;
}

}  // extern "C"
