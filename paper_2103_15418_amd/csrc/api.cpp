// C ABI of liblpf: configuration, workspace carving, call-order checks and
// the per-step orchestration of the device kernels.  No arithmetic of the
// method runs here; every stage is a kernel on the context's stream.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lpf_internal.h"

namespace lpf {
hipError_t launch_windows_gather(lpf_ctx* c, int n, const int32_t* d_slots, const int64_t* d_tend,
                                 float* d_out, hipStream_t s);
hipError_t launch_ended_ends(lpf_ctx* c, int32_t* slots_out, int64_t* tend_out);
hipError_t cnn_forward(const lpf_model* m, const float* windows, const int* n_dev, int n_cap, float* mu,
                       float* L, hipStream_t s);
hipError_t launch_gather_ended(lpf_ctx* c, int ci, int32_t* hdr, float* out, int32_t* rows, int cap,
                               hipStream_t s, bool first);
hipError_t cnn_forward_static(const lpf_model* m, const float* windows, int n, float* mu, float* L, hipStream_t s);
int static_max_windows();
float* model_window_buffer(const lpf_model* m);
float* model_mu_buffer(const lpf_model* m);
float* model_L_buffer(const lpf_model* m);
int model_max_batch(const lpf_model* m);
float* model_host_rows(const lpf_model* m, size_t n);
size_t model_blob_bytes();
int model_workspace_size(int precision, int maxb, size_t* bytes);
int model_create(const void* weights, size_t bytes, int precision, int maxb, void* ws, size_t ws_bytes,
                 hipStream_t s, lpf_model** out);
void model_destroy(lpf_model* m);

namespace {

constexpr size_t kAlign = 256;

struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + kAlign - 1) & ~(kAlign - 1);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

int validate(const lpf_config* c, std::string* why) {
    auto bad = [&](const char* m) {
        if (why) *why = m;
        return LPF_EINVAL;
    };
    if (!c) return bad("null config");
    if (c->B < 1 || c->B > kMaxB) return bad("B must be in 1..16");
    if (c->H < 1 || c->H > kMaxDim || c->W < 1 || c->W > kMaxDim) return bad("H, W must be in 1..4096");
    if (!(c->kappa >= 0.0f) || !std::isfinite(c->kappa)) return bad("kappa must be finite and >= 0");
    if (c->kernel != LPF_KERNEL_GAUSS && c->kernel != LPF_KERNEL_BOX && c->kernel != LPF_KERNEL_DISK)
        return bad("unknown kernel");
    if (c->kernel == LPF_KERNEL_GAUSS && !(c->bg_sigma > 0.0f)) return bad("bg_sigma must be > 0");
    int k = c->bg_halfwidth > 0 ? c->bg_halfwidth : (int)std::ceil(3.0 * (double)c->bg_sigma);
    if (k < 1 || k > kMaxK) return bad("background half-width must be in 1..40");
    if (c->kernel == LPF_KERNEL_DISK &&
        (k > disk_max_halfwidth() || c->clip_iters != 1 || c->filter_precision != LPF_PREC_FP32))
        return bad("the disk kernel needs radius <= 32, clip_iters = 1 and float32 filters");
    if (!(c->psf_sigma >= 0.0f) || !std::isfinite(c->psf_sigma)) return bad("psf_sigma must be finite and >= 0");
    if (c->psf_sigma > 0.0f) {
        const int kp = c->psf_halfwidth > 0 ? c->psf_halfwidth : (int)std::ceil(4.0 * (double)c->psf_sigma);
        if (kp < 1 || kp > kMaxK) return bad("PSF half-width must be in 1..40");
        if (c->filter_precision != LPF_PREC_FP32) return bad("the PSF pre-filter needs float32 filters");
    }
    if (c->flux_bg_width < 0 || c->flux_bg_width > 16) return bad("flux_bg_width in 0..16");
    if (c->clip_iters < 1 || c->clip_iters > kMaxIters) return bad("clip_iters must be in 1..16");
    if (c->peak_halfwidth < 1 || c->peak_halfwidth > kMaxPeakK) return bad("peak_halfwidth in 1..8");
    if (c->flux_halfwidth < 0 || c->flux_halfwidth > kMaxFluxK) return bad("flux_halfwidth in 0..8");
    if (!(c->dup_radius >= 0.0f) || !(c->assoc_radius >= 0.0f)) return bad("radii must be >= 0");
    if (c->monitor_steps < 0) return bad("monitor_steps must be >= 0");
    if (c->backfill_steps < 0 || c->backfill_steps > 4096) return bad("backfill_steps in 0..4096");
    if (c->ring_len != kRing) return bad("ring_len must be 64");
    if (!(c->qc_band_z > 0.0f)) return bad("qc_band_z must be > 0");
    if (!(c->qc_rms_floor >= 0.0f)) return bad("qc_rms_floor must be >= 0");
    if (!(c->qc_pixel_zeta > 0.0f)) return bad("qc_pixel_zeta must be > 0");
    if (c->qc_warmup < 0) return bad("qc_warmup must be >= 0");
    if (c->max_sources < 1 || c->max_sources > kMaxSources) return bad("max_sources in 1..65536");
    if (c->peak_cap < 1 || (int64_t)c->peak_cap * c->B > kCatMaxPeaks) return bad("B * peak_cap must be <= 8192");
    if (c->filter_precision != LPF_PREC_FP32 && c->filter_precision != LPF_PREC_BF16 &&
        c->filter_precision != LPF_PREC_FP16)
        return bad("unknown filter_precision");
    if (c->filter_precision != LPF_PREC_FP32 &&
        (c->clip_iters != 1 || c->W % 4 != 0 || (k != 15 && k != 24 && k != 36)))
        return bad("16-bit filters need clip_iters = 1, W % 4 = 0 and half-width 15, 24 or 36");
    if (c->pipeline_ingest != 0 && c->pipeline_ingest != 1) return bad("pipeline_ingest must be 0 or 1");
    if (c->grid_rows) {
        bool used[kGridRows] = {};
        for (int b = 0; b < c->B; ++b) {
            int r = c->grid_rows[b];
            if (r < 0 || r >= kGridRows || used[r]) return bad("grid_rows must be distinct rows in 0..15");
            used[r] = true;
        }
    }
    return LPF_OK;
}

Derived derive(const lpf_config* c) {
    Derived d{};
    d.k = c->bg_halfwidth > 0 ? c->bg_halfwidth : (int)std::ceil(3.0 * (double)c->bg_sigma);
    // the cache holds the backfill window and the current step, and with a
    // pipelined ingest also the next step, written while this one is measured
    d.Tc = c->backfill_steps + 1 + (c->pipeline_ingest ? 1 : 0);
    d.HW = (size_t)c->H * c->W;
    d.plane = (size_t)c->B * d.HW;
    d.masked = c->sky_mask != nullptr;
    d.dyn = c->clip_iters > 1 || c->debug_planes != 0;
    d.mwords = (c->W + 31) / 32;
    d.disk = c->kernel == LPF_KERNEL_DISK;
    d.strip = !d.disk && c->W % 4 == 0 && (d.k == 15 || d.k == 24 || d.k == 36);
    d.pre = c->psf_sigma > 0.0f;
    d.kpsf = d.pre ? (c->psf_halfwidth > 0 ? c->psf_halfwidth : (int)std::ceil(4.0 * (double)c->psf_sigma)) : 0;
    // ~32K pixels per ingest workgroup (one partial sum each): 512 workgroups
    // for 16 x 1024^2.  Beside the catalogue (pipelined ingest) the step
    // measured 0.344 ms with 8K-pixel blocks, 0.321 with 32K and 0.337 with
    // 64K; the block size also fixes the partial sums, so the sequential and
    // the pipelined ingest share it and stay bitwise equal
    size_t nb = (d.HW + 32767) / 32768;
    if (nb < 1) nb = 1;
    d.nblk = (int)nb;
    return d;
}

// Carves every device buffer; with base == nullptr only sizes the total.
size_t carve(const lpf_config* c, const Derived& d, char* base, DevBufs* b) {
    Carver cv{base};
    const size_t S = (size_t)c->max_sources;
    b->cache = cv.take<float>((size_t)d.Tc * d.plane);
    b->cache_t = cv.take<int64_t>(d.Tc);
    b->cache_rej = cv.take<uint32_t>(d.Tc);
    b->wf_mean = cv.take<float>(2 * d.plane);
    b->wf_m2 = cv.take<float>(2 * d.plane);
    b->wf_n = cv.take<int32_t>(kMaxB);
    b->wf_cur = cv.take<int32_t>(kMaxB);
    b->mask = cv.take<uint8_t>(d.HW);
    b->mask_bits = cv.take<uint32_t>((size_t)c->H * d.mwords);
    b->inv_den = cv.take<float>(d.HW);
    b->centre = cv.take<float>(d.plane);
    b->resid = d.strip ? cv.take<float>(d.plane) : nullptr;
    b->spread = d.dyn ? cv.take<float>(d.plane) : nullptr;
    b->clip = d.dyn ? cv.take<uint8_t>(2 * d.plane) : nullptr;
    b->den = c->clip_iters > 1 ? cv.take<float>(d.plane) : nullptr;
    b->partials = cv.take<BandPartial>((size_t)c->B * d.nblk);
    b->bandstats = cv.take<double>(6 * kMaxB);
    b->changed = cv.take<int32_t>((kMaxIters + 1) * kMaxB);
    b->peak_cnt = cv.take<int32_t>(kMaxB);
    b->cand = (d.strip || d.disk) ? cv.take<int2>(d.plane) : nullptr;
    b->cand_cnt = cv.take<int32_t>(kMaxB);
    b->peak_raw = cv.take<PeakRec>((size_t)c->B * c->peak_cap);
    b->peak_sorted = cv.take<PeakRec>((size_t)c->B * c->peak_cap);
    b->cat_dec = cv.take<int32_t>(kCatMaxPeaks);
    b->cat_order = cv.take<int32_t>(kCatMaxPeaks);
    b->cat_kept = cv.take<int32_t>(kCatMaxPeaks);
    b->cat_nbr = cv.take<int32_t>((size_t)kCatMaxPeaks * (kNbr + 1));
    b->cat_cand = cv.take<int32_t>((size_t)kCatMaxPeaks * (kCand + 1));
    b->cat_gkeys = cv.take<uint64_t>(kCatMaxPeaks);
    b->cat_gpos = cv.take<int32_t>(kCatMaxPeaks);
    b->cat_gflag = cv.take<uint8_t>(kCatMaxPeaks);
    b->cat_live = cv.take<int32_t>(S);
    b->cat_lpos = cv.take<int32_t>(S);
    b->cat_taken = cv.take<uint32_t>((S + 31) / 32);
    b->cat_seen = cv.take<uint32_t>((S + 31) / 32);
    b->cat_rowoff = cv.take<int32_t>((size_t)c->H + 1);
    b->cat_rowcur = cv.take<int32_t>((size_t)c->H);
    b->cat_rowidx = cv.take<int32_t>(kCatMaxPeaks);
    b->cat_lrowidx = cv.take<int32_t>(S);
    b->free_list = cv.take<int32_t>(S);
    b->src_id = cv.take<int32_t>(S);
    b->src_row = cv.take<int32_t>(S);
    b->src_col = cv.take<int32_t>(S);
    b->src_state = cv.take<int32_t>(S);
    b->src_tfirst = cv.take<int64_t>(S);
    b->src_tlast = cv.take<int64_t>(S);
    b->src_tend = cv.take<int64_t>(S);
    b->src_new = cv.take<int32_t>(S);
    b->list_measured = cv.take<int2>(S);
    b->list_new = cv.take<int2>(S);
    b->list_ended = cv.take<int32_t>(S);
    b->ring = cv.take<float>(S * c->B * kRing);
    b->ring_t = cv.take<int64_t>(S * kRing);
    b->ring_v = cv.take<uint32_t>(S * kRing);
    b->status = cv.take<DevStatus>(1);
    b->events = cv.take<lpf_source>(2 * S);
    b->infer_slots = cv.take<int32_t>(S);
    b->infer_tend = cv.take<int64_t>(S);
    b->pre = d.pre ? cv.take<float>(d.plane) : nullptr;
    b->inv_den_psf = d.pre ? cv.take<float>(d.HW) : nullptr;
    b->cutout = cv.take<float>((size_t)d.Tc * c->B * (2 * kMaxCutoutHalf + 1) * (2 * kMaxCutoutHalf + 1));
    return (cv.off + kAlign - 1) & ~(kAlign - 1);
}

int fail(lpf_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int dev_fail(lpf_ctx* c, hipError_t e, const char* where) {
    if (c) {
        c->poisoned = true;
        c->err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return LPF_EDEVICE;
}

#define LPF_CHECK_CTX(c)                                   \
    do {                                                   \
        if (!(c)) return LPF_EINVAL;                       \
        if ((c)->poisoned) return LPF_EDEVICE;             \
    } while (0)

#define LPF_HIP(c, expr, where)                            \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return dev_fail((c), _e, (where)); \
    } while (0)

int pmod(int64_t a, int m) {
    int64_t r = a % m;
    return (int)(r < 0 ? r + m : r);
}

// Events that order kernels after kernels on one device's streams (never
// waited on by the host, never ordering a copy): no timing and no system-scope
// fence, so a record costs no cache maintenance for host visibility.
constexpr unsigned kDevEvent = hipEventDisableTiming | hipEventDisableSystemFence;

// Waits for every stream of a context (before host reads of its state).
hipError_t sync_all(lpf_ctx* c) {
    hipError_t e;
    if (c->ing_stream && (e = hipStreamSynchronize(c->ing_stream)) != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}


}  // namespace
namespace {

// The network on a gathered ticket's windows, on the model's stream after
// event `after`, then the copy of its result block to the ticket's pinned slot.
int launch_ticket(lpf_model* m, int slot, hipEvent_t after, lpf_ctx* c0) {
    hipStream_t s = m->istream;
    const CnnWork& w = m->work;
    int32_t* hdr = w.sblk[slot];
    float* mu = reinterpret_cast<float*>(hdr + 4 + 2 * (size_t)m->max_batch);
    float* L = mu + 4 * (size_t)m->max_batch;
    LPF_HIP(c0, hipStreamWaitEvent(s, after, 0), "event wait");
    {
        StageTimer tm(c0, 6, s);
        LPF_HIP(c0, cnn_forward(m, w.swin[slot], hdr, m->max_batch, mu, L, s), "cnn");
    }
    LPF_HIP(c0, hipMemcpyAsync(m->h_res[slot], hdr, w.out_bytes, hipMemcpyDeviceToHost, s), "result D2H");
    LPF_HIP(c0, hipEventRecord(m->ev_done[slot], s), "event record");
    return LPF_OK;
}

// Issues a context's deferred launch: after `after`, or after all the work on
// the context's stream so far (its gather included).  The gather itself
// records no event: the detect that usually issues the launch passes one it
// records anyway, and an event record costs the stream a few microseconds.
int flush_pending(lpf_ctx* c, hipEvent_t after) {
    lpf_model* m = c->pend_model;
    if (!m) return LPF_OK;
    const int slot = c->pend_slot;
    c->pend_model = nullptr;
    c->pend_slot = -1;
    m->pend_ctx[slot] = nullptr;
    if (!after) {
        LPF_HIP(c, hipEventRecord(m->ev_gath[slot], c->stream), "event record");
        after = m->ev_gath[slot];
    }
    return launch_ticket(m, slot, after, c);
}

}  // namespace

// 1 when the results of an asynchronous ticket are on the host, 0 if not yet,
// negative on error or for an unknown ticket (serving loop).
int ticket_state(lpf_model* m, int64_t ticket) {
    const int slot = (int)(ticket % kInflight);
    if (ticket < 0 || m->slot_ticket[slot] != ticket) return LPF_EINVAL;
    if (m->pend_ctx[slot]) return 0;
    const hipError_t q = hipEventQuery(m->ev_done[slot]);
    if (q == hipSuccess) return 1;
    return q == hipErrorNotReady ? 0 : LPF_EDEVICE;
}

// Peaks and events of a context's last detect, as lpf_detect returns them
// (ended episodes sorted by id); synchronises (serving loop, record mode).
int read_last_lists(lpf_ctx* c, std::vector<lpf_peak>* peaks, std::vector<lpf_source>* events) {
    DevStatus st;
    LPF_HIP(c, hipMemcpyAsync(&st, c->buf.status, sizeof(st), hipMemcpyDeviceToHost, c->stream), "status D2H");
    LPF_HIP(c, hipStreamSynchronize(c->stream), "lists sync");
    peaks->resize(std::max(st.n_peaks, 0));
    if (!peaks->empty())
        LPF_HIP(c, hipMemcpy(peaks->data(), c->buf.peak_sorted, peaks->size() * sizeof(lpf_peak),
                             hipMemcpyDeviceToHost), "peaks D2H");
    const int nev = std::max(st.n_new + st.n_ended, 0);
    events->resize(nev);
    if (nev > 0)
        LPF_HIP(c, hipMemcpy(events->data(), c->buf.events, nev * sizeof(lpf_source), hipMemcpyDeviceToHost),
                "events D2H");
    std::sort(events->begin() + std::min(st.n_new, nev), events->end(),
              [](const lpf_source& a, const lpf_source& b) { return a.id < b.id; });
    return LPF_OK;
}

}  // namespace lpf

using namespace lpf;

extern "C" {

int lpf_config_default(lpf_config* c, int32_t B, int32_t H, int32_t W) {
    if (!c) return LPF_EINVAL;
    std::memset(c, 0, sizeof(*c));
    c->B = B;
    c->H = H;
    c->W = W;
    c->sky_mask = nullptr;
    c->grid_rows = nullptr;
    c->kappa = 4.5f;
    c->bg_sigma = 8.0f;
    c->bg_halfwidth = 0;
    c->kernel = LPF_KERNEL_GAUSS;
    c->clip_iters = 1;
    c->peak_halfwidth = 3;
    c->flux_halfwidth = 2;
    c->dup_radius = 3.0f;
    c->assoc_radius = 3.0f;
    c->monitor_steps = 31;
    c->backfill_steps = 32;
    c->ring_len = kRing;
    c->qc_band_z = 5.0f;
    c->qc_rms_z = 5.0f;
    c->qc_rms_floor = 0.05f;
    c->qc_pixel_zeta = 30.0f;
    c->qc_warmup = 8;
    c->max_sources = 8192;
    c->peak_cap = 512;
    c->filter_precision = LPF_PREC_FP32;
    c->debug_planes = 0;
    c->psf_sigma = 0.0f;
    c->psf_halfwidth = 0;
    c->flux_bg_width = 0;
    return LPF_OK;
}

int lpf_workspace_size(const lpf_config* cfg, size_t* bytes) {
    if (!bytes) return LPF_EINVAL;
    int rc = validate(cfg, nullptr);
    if (rc != LPF_OK) return rc;
    Derived d = derive(cfg);
    DevBufs b{};
    *bytes = carve(cfg, d, nullptr, &b);
    return LPF_OK;
}

int lpf_create(const lpf_config* cfg, void* ws, size_t bytes, void* stream, lpf_ctx** out) {
    if (!out) return LPF_EINVAL;
    *out = nullptr;
    std::string why;
    int rc = validate(cfg, &why);
    if (rc != LPF_OK) return rc;
    if (!ws) return LPF_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return LPF_EINVAL;
    Derived d = derive(cfg);
    DevBufs tmp{};
    const size_t need = carve(cfg, d, nullptr, &tmp);
    if (bytes < need) return LPF_ENOMEM;
    lpf_ctx* c = new (std::nothrow) lpf_ctx();
    if (!c) return LPF_ENOMEM;
    c->cfg = *cfg;
    c->cfg.sky_mask = nullptr;
    c->cfg.grid_rows = nullptr;
    c->d = d;
    c->stream = static_cast<hipStream_t>(stream);
    c->t_last = INT64_MIN;
    c->t_start = INT64_MIN;
    c->n_frames = 0;
    c->phase = 0;
    c->poisoned = false;
    for (int b = 0; b < cfg->B; ++b) c->grid_rows[b] = cfg->grid_rows ? cfg->grid_rows[b] : b * (kGridRows / cfg->B);
    // taps: g_u = exp(-u^2 / 2 s^2) / sum_v exp(-v^2 / 2 s^2), or 1 / (2k+1)
    {
        std::memset(&c->taps, 0, sizeof(c->taps));
        c->taps.k = d.k;
        double sum = 0.0, e[2 * kMaxK + 1];
        for (int u = -d.k; u <= d.k; ++u) {
            double v = cfg->kernel == LPF_KERNEL_BOX ? 1.0
                                                     : std::exp(-(double)u * u / (2.0 * (double)cfg->bg_sigma * cfg->bg_sigma));
            e[u + d.k] = v;
            sum += v;
        }
        for (int i = 0; i <= 2 * d.k; ++i) c->taps.g[i] = (float)(e[i] / sum);
    }
    // PSF pre-filter taps: Gaussian of width psf_sigma normalised over [-kpsf, kpsf]
    std::memset(&c->taps_psf, 0, sizeof(c->taps_psf));
    if (d.pre) {
        c->taps_psf.k = d.kpsf;
        double sum = 0.0, e[2 * kMaxK + 1];
        for (int u = -d.kpsf; u <= d.kpsf; ++u) {
            e[u + d.kpsf] = std::exp(-(double)u * u / (2.0 * (double)cfg->psf_sigma * cfg->psf_sigma));
            sum += e[u + d.kpsf];
        }
        for (int i = 0; i <= 2 * d.kpsf; ++i) c->taps_psf.g[i] = (float)(e[i] / sum);
    }
    carve(cfg, d, static_cast<char*>(ws), &c->buf);
    hipStream_t s = c->stream;
    auto zero = [&](void* p, size_t n) { return p ? hipMemsetAsync(p, 0, n, s) : hipSuccess; };
    hipError_t e = hipSuccess;
    if (d.masked) e = hipMemcpyAsync(c->buf.mask, cfg->sky_mask, d.HW, hipMemcpyHostToDevice, s);
    else e = hipMemsetAsync(c->buf.mask, 1, d.HW, s);
    if (e == hipSuccess) e = zero(c->buf.wf_mean, 2 * d.plane * sizeof(float));
    if (e == hipSuccess) e = zero(c->buf.wf_m2, 2 * d.plane * sizeof(float));
    if (e == hipSuccess) e = zero(c->buf.wf_n, kMaxB * sizeof(int32_t));
    if (e == hipSuccess) e = zero(c->buf.wf_cur, kMaxB * sizeof(int32_t));
    if (e == hipSuccess) e = zero(c->buf.centre, d.plane * sizeof(float));
    if (e == hipSuccess && c->buf.spread) e = zero(c->buf.spread, d.plane * sizeof(float));
    if (e == hipSuccess && c->buf.clip) e = zero(c->buf.clip, 2 * d.plane);
    if (e == hipSuccess) e = zero(c->buf.src_id, cfg->max_sources * sizeof(int32_t));
    // detection counters (cleared again by the catalogue kernel of every step)
    if (e == hipSuccess) e = zero(c->buf.peak_cnt, kMaxB * sizeof(int32_t));
    if (e == hipSuccess) e = zero(c->buf.cand_cnt, kMaxB * sizeof(int32_t));
    if (e == hipSuccess) e = zero(c->buf.changed, (size_t)(kMaxIters + 1) * kMaxB * sizeof(int32_t));
    if (e == hipSuccess) e = launch_table_init(c);
    if (e == hipSuccess) e = launch_pack_mask(c);
    if (e == hipSuccess) e = d.disk ? launch_disk_inv_den(c) : launch_inv_den(c);
    if (e == hipSuccess && cfg->pipeline_ingest) {
        e = hipStreamCreateWithFlags(&c->ing_stream, hipStreamNonBlocking);   // default priority
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_filt, kDevEvent);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_qc, kDevEvent);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_centre, kDevEvent);
    }
    if (e == hipSuccess && (d.masked || cfg->pipeline_ingest)) {
        // mask copy is from pageable host memory, and a pipelined ingest is
        // not ordered after this initialisation: finish before returning
        e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) {
        dev_fail(c, e, "lpf_create");
        lpf_destroy(c);
        return LPF_EDEVICE;
    }
    *out = c;
    return LPF_OK;
}

void lpf_destroy(lpf_ctx* c) {
    if (!c) return;
    if (!c->poisoned) (void)flush_pending(c, nullptr);   // its ticket stays collectible
    if (c->pend_model) {
        c->pend_model->pend_ctx[c->pend_slot] = nullptr;
        c->pend_model = nullptr;
    }
    if (!c->poisoned) (void)sync_all(c);
    for (auto& e : c->prof_pool) (void)hipEventDestroy(e);
    if (c->ev_ready) (void)hipEventDestroy(c->ev_ready);
    if (c->ev_filt) (void)hipEventDestroy(c->ev_filt);
    if (c->ev_qc) (void)hipEventDestroy(c->ev_qc);
    if (c->ev_centre) (void)hipEventDestroy(c->ev_centre);
    if (c->ing_stream) (void)hipStreamDestroy(c->ing_stream);
    delete c;
}

int lpf_ingest_frame(lpf_ctx* c, int64_t t, const float* cube, int32_t on_device, uint32_t* rej_out) {
    LPF_CHECK_CTX(c);
    if (!cube) return fail(c, LPF_EINVAL, "null cube");
    if (c->phase == 1 || c->phase == 2) return fail(c, LPF_ESTATE, "ingest before detect/extract_flux finished");
    if (c->n_frames > 0 && t <= c->t_last) return fail(c, LPF_EORDER, "t must increase");
    const int slot = pmod(t, c->d.Tc);
    float* dst = c->buf.cache + (size_t)slot * c->d.plane;
    // pipelined: the context's own ingest stream, ordered after the previous
    // step's filters (which follow the flux that last read this cache slot:
    // the cache holds backfill_steps + 2 steps and a flux reads back
    // backfill_steps), or after everything on the context's stream before
    // the first detect or when t skips a step (then the flux just enqueued
    // may read the slot this frame overwrites)
    hipStream_t s = c->ing_stream ? c->ing_stream : c->stream;
    if (c->ing_stream) {
        if (!c->filt_recorded || (c->n_frames > 0 && t - c->t_last >= 2))
            LPF_HIP(c, hipEventRecord(c->ev_filt, c->stream), "event record");
        LPF_HIP(c, hipStreamWaitEvent(s, c->ev_filt, 0), "event wait");
    }
    if (on_device) {
        StageTimer tm(c, 0, s);
        LPF_HIP(c, launch_ingest(c, cube, true, slot, s), "ingest");
    } else {
        LPF_HIP(c, hipMemcpyAsync(dst, cube, c->d.plane * sizeof(float), hipMemcpyHostToDevice, s),
                "ingest H2D");
        StageTimer tm(c, 0, s);
        LPF_HIP(c, launch_ingest(c, dst, false, slot, s), "ingest");
    }
    {
        StageTimer tm(c, 1, s);
        LPF_HIP(c, launch_qc_decide(c, slot, t, s), "qc");
    }
    if (c->ing_stream) {
        LPF_HIP(c, hipEventRecord(c->ev_qc, s), "event record");
        c->qc_pending = true;
    }
    if (!on_device) LPF_HIP(c, hipStreamSynchronize(s), "ingest sync");
    if (c->n_frames == 0) c->t_start = t;
    c->t_last = t;
    c->n_frames++;
    c->phase = 1;
    c->host_n_ended = -1;
    if (rej_out) {
        uint32_t r = 0;
        LPF_HIP(c, hipMemcpyAsync(&r, &c->buf.status->rejected, sizeof(r), hipMemcpyDeviceToHost, s),
                "ingest D2H");
        LPF_HIP(c, hipStreamSynchronize(s), "ingest sync");
        *rej_out = r;
    }
    return LPF_OK;
}

int lpf_detect(lpf_ctx* c, lpf_peak* peaks, int32_t cap, int32_t* n_peaks, lpf_source* events,
               int32_t ev_cap, int32_t* n_events) {
    LPF_CHECK_CTX(c);
    if (c->phase != 1) return fail(c, LPF_ESTATE, "detect needs a fresh ingest");
    const int slot = pmod(c->t_last, c->d.Tc);
    // (the detection counters were cleared by the previous step's catalogue)
    if (c->qc_pending) {
        LPF_HIP(c, hipStreamWaitEvent(c->stream, c->ev_qc, 0), "event wait");
        c->qc_pending = false;
    }
    LPF_HIP(c, launch_filters(c, slot), "filters");
    if (c->ing_stream) {
        // the next ingest may start now: it writes a cache slot nothing of
        // this step reads, and state the catalogue and flux do not touch
        LPF_HIP(c, hipEventRecord(c->ev_filt, c->stream), "event record");
        c->filt_recorded = true;
        // the network of the previous step's ticket runs beside this step's
        // spread pass and catalogue (launched after the centre pass)
        const int rc = flush_pending(c, c->ev_centre);
        if (rc != LPF_OK) return rc;
    }
    {
        StageTimer tm(c, 4);
        LPF_HIP(c, launch_catalog(c, c->t_last), "catalog");
    }
    c->phase = 2;
    const bool want = peaks || n_peaks || events || n_events;
    if (!want) return LPF_OK;
    DevStatus st;
    LPF_HIP(c, hipMemcpyAsync(&st, c->buf.status, sizeof(st), hipMemcpyDeviceToHost, c->stream), "detect D2H");
    LPF_HIP(c, hipStreamSynchronize(c->stream), "detect sync");
    c->host_n_ended = st.n_ended;
    if (n_peaks) *n_peaks = st.n_peaks;
    if (peaks && cap > 0 && st.n_peaks > 0) {
        const int n = std::min(cap, st.n_peaks);
        LPF_HIP(c, hipMemcpy(peaks, c->buf.peak_sorted, n * sizeof(lpf_peak), hipMemcpyDeviceToHost), "peaks D2H");
    }
    const int nev = st.n_new + st.n_ended;
    if (n_events) *n_events = nev;
    if (events && ev_cap > 0 && nev > 0) {
        std::vector<lpf_source> tmp(nev);
        LPF_HIP(c, hipMemcpy(tmp.data(), c->buf.events, nev * sizeof(lpf_source), hipMemcpyDeviceToHost),
                "events D2H");
        c->host_ended_ids.resize(st.n_ended);
        for (int k = 0; k < st.n_ended; ++k) c->host_ended_ids[k] = tmp[st.n_new + k].id;
        std::sort(tmp.begin() + st.n_new, tmp.end(),
                  [](const lpf_source& a, const lpf_source& b) { return a.id < b.id; });
        std::memcpy(events, tmp.data(), std::min(ev_cap, nev) * sizeof(lpf_source));
    } else {
        c->host_ended_ids.clear();
        if (st.n_ended > 0) c->host_n_ended = -1;   // ids not read: inference reads them itself
    }
    if (st.overflow_bands || st.n_dropped) return fail(c, LPF_EFULL, "peak or source capacity reached");
    return LPF_OK;
}

int lpf_extract_flux(lpf_ctx* c) {
    LPF_CHECK_CTX(c);
    if (c->phase != 2) return fail(c, LPF_ESTATE, "extract_flux needs detect first");
    {
        StageTimer tm(c, 5);
        LPF_HIP(c, launch_flux(c, pmod(c->t_last, c->d.Tc), c->t_last), "flux");
    }
    c->phase = 3;
    return LPF_OK;
}

// ---- batch forms: grouped launches over several contexts --------------------

namespace {

// Common checks of a batch call: distinct, healthy contexts on one stream,
// none with a pipelined ingest.  Returns the shared stream through *s.
int batch_check(lpf_ctx* const* cs, int32_t n, hipStream_t* s) {
    if (!cs || n < 1) return LPF_EINVAL;
    for (int i = 0; i < n; ++i) {
        LPF_CHECK_CTX(cs[i]);
        if (cs[i]->stream != cs[0]->stream) return fail(cs[i], LPF_EINVAL, "batch contexts must share one stream");
        if (cs[i]->ing_stream) return fail(cs[i], LPF_EINVAL, "batch calls need pipeline_ingest = 0");
        for (int j = 0; j < i; ++j)
            if (cs[j] == cs[i]) return fail(cs[i], LPF_EINVAL, "context repeated in a batch");
    }
    *s = cs[0]->stream;
    return LPF_OK;
}

}  // namespace

int lpf_ingest_batch(lpf_ctx* const* cs, const int64_t* t, const float* const* cubes, int32_t on_device,
                     int32_t n) {
    hipStream_t s = nullptr;
    int rc = batch_check(cs, n, &s);
    if (rc != LPF_OK) return rc;
    if (!t || !cubes) return fail(cs[0], LPF_EINVAL, "null t or cubes");
    for (int i = 0; i < n; ++i) {
        lpf_ctx* c = cs[i];
        if (!cubes[i]) return fail(c, LPF_EINVAL, "null cube");
        if (c->phase == 1 || c->phase == 2) return fail(c, LPF_ESTATE, "ingest before detect/extract_flux finished");
        if (c->n_frames > 0 && t[i] <= c->t_last) return fail(c, LPF_EORDER, "t must increase");
    }
    std::vector<int> slots(n);
    std::vector<const float*> srcs(n);
    for (int i = 0; i < n; ++i) {
        lpf_ctx* c = cs[i];
        slots[i] = pmod(t[i], c->d.Tc);
        float* dst = c->buf.cache + (size_t)slots[i] * c->d.plane;
        if (on_device) {
            srcs[i] = cubes[i];
        } else {
            LPF_HIP(c, hipMemcpyAsync(dst, cubes[i], c->d.plane * sizeof(float), hipMemcpyHostToDevice, s),
                    "ingest H2D");
            srcs[i] = dst;
        }
    }
    // grouped ingest passes (contexts with and without float4-aligned planes apart),
    // then grouped QC decisions
    for (int vec = 0; vec < 2; ++vec) {
        std::vector<lpf_ctx*> gc;
        std::vector<const float*> gs;
        std::vector<int> gl;
        for (int i = 0; i < n; ++i) {
            if ((int)((cs[i]->d.HW % 4) == 0) != vec) continue;
            gc.push_back(cs[i]);
            gs.push_back(srcs[i]);
            gl.push_back(slots[i]);
        }
        for (size_t k = 0; k < gc.size(); k += kGroupMax) {
            const int m = (int)std::min<size_t>(kGroupMax, gc.size() - k);
            LPF_HIP(gc[k], launch_ingest_group(gc.data() + k, gs.data() + k, gl.data() + k, m, on_device != 0,
                                               vec != 0, s), "ingest");
        }
    }
    for (int k = 0; k < n; k += kGroupMax) {
        const int m = std::min(kGroupMax, n - k);
        LPF_HIP(cs[k], launch_qc_decide_group(cs + k, slots.data() + k, t + k, m, s), "qc");
    }
    if (!on_device) LPF_HIP(cs[0], hipStreamSynchronize(s), "ingest sync");
    for (int i = 0; i < n; ++i) {
        lpf_ctx* c = cs[i];
        if (c->n_frames == 0) c->t_start = t[i];
        c->t_last = t[i];
        c->n_frames++;
        c->phase = 1;
        c->host_n_ended = -1;
    }
    return LPF_OK;
}

int lpf_detect_batch(lpf_ctx* const* cs, int32_t n) {
    hipStream_t s = nullptr;
    int rc = batch_check(cs, n, &s);
    if (rc != LPF_OK) return rc;
    for (int i = 0; i < n; ++i)
        if (cs[i]->phase != 1) return fail(cs[i], LPF_ESTATE, "detect needs a fresh ingest");
    // filters: classes of groupable contexts share launches; the others run alone
    std::vector<char> done(n, 0);
    for (int i = 0; i < n; ++i) {
        if (done[i]) continue;
        std::vector<lpf_ctx*> gc;
        std::vector<int> gl;
        for (int j = i; j < n; ++j) {
            if (done[j] || !filters_groupable(cs[i], cs[j])) continue;
            done[j] = 1;
            gc.push_back(cs[j]);
            gl.push_back(pmod(cs[j]->t_last, cs[j]->d.Tc));
        }
        if (gc.empty()) {
            done[i] = 1;
            LPF_HIP(cs[i], launch_filters(cs[i], pmod(cs[i]->t_last, cs[i]->d.Tc)), "filters");
            continue;
        }
        for (size_t k = 0; k < gc.size(); k += kGroupMax) {
            const int m = (int)std::min<size_t>(kGroupMax, gc.size() - k);
            LPF_HIP(gc[k], launch_filters_group(gc.data() + k, gl.data() + k, m, s), "filters");
        }
    }
    std::vector<int64_t> ts(n);
    for (int i = 0; i < n; ++i) ts[i] = cs[i]->t_last;
    for (int k = 0; k < n; k += kGroupMax) {
        const int m = std::min(kGroupMax, n - k);
        LPF_HIP(cs[k], launch_catalog_group(cs + k, ts.data() + k, m, s), "catalog");
    }
    for (int i = 0; i < n; ++i) cs[i]->phase = 2;
    return LPF_OK;
}

int lpf_extract_flux_batch(lpf_ctx* const* cs, int32_t n) {
    hipStream_t s = nullptr;
    int rc = batch_check(cs, n, &s);
    if (rc != LPF_OK) return rc;
    for (int i = 0; i < n; ++i)
        if (cs[i]->phase != 2) return fail(cs[i], LPF_ESTATE, "extract_flux needs detect first");
    std::vector<int64_t> ts(n);
    for (int i = 0; i < n; ++i) ts[i] = cs[i]->t_last;
    for (int k = 0; k < n; k += kGroupMax) {
        const int m = std::min(kGroupMax, n - k);
        LPF_HIP(cs[k], launch_flux_group(cs + k, ts.data() + k, m, s), "flux");
    }
    for (int i = 0; i < n; ++i) cs[i]->phase = 3;
    return LPF_OK;
}

// ---- candidate selection and image cutouts (Sec. 2.3.1, Sec. 3.3-3.4) ---------

int lpf_select_candidates(const float* mu, const float* L, int32_t n, float dm_min, float sigma_max,
                          int32_t* idx_out, float* sigma_out, int32_t* n_out) {
    if (n < 0 || !n_out || (n > 0 && (!mu || !L || !idx_out))) return LPF_EINVAL;
    // Sigma = L L^T with L packed row by row: Sigma_00 = L_00^2, so sigma_DM = |L_00|
    std::vector<int32_t> keep;
    for (int i = 0; i < n; ++i) {
        const float sg = std::fabs(L[(size_t)i * 10]);
        if (sigma_out) sigma_out[i] = sg;
        if (mu[(size_t)i * 4] > dm_min && sg <= sigma_max) keep.push_back(i);
    }
    std::stable_sort(keep.begin(), keep.end(),
                     [&](int32_t a, int32_t b) { return std::fabs(L[(size_t)a * 10]) < std::fabs(L[(size_t)b * 10]); });
    std::copy(keep.begin(), keep.end(), idx_out);
    *n_out = (int32_t)keep.size();
    return LPF_OK;
}

int lpf_read_cutouts(lpf_ctx* c, int32_t row, int32_t col, int32_t half, int64_t t_first, int32_t n_steps,
                     float* out, uint8_t* have) {
    LPF_CHECK_CTX(c);
    if (!out || half < 0 || half > kMaxCutoutHalf || n_steps < 1 || n_steps > c->d.Tc)
        return fail(c, LPF_EINVAL, "cutout: half in 0..32, 1 <= n_steps <= cache depth, out non-null");
    LPF_HIP(c, sync_all(c), "cutout sync");
    LPF_HIP(c, launch_cutouts(c, row, col, half, t_first, n_steps), "cutout");
    const size_t side = (size_t)(2 * half + 1);
    const size_t nval = (size_t)n_steps * c->cfg.B * side * side;
    LPF_HIP(c, hipMemcpyAsync(out, c->buf.cutout, nval * sizeof(float), hipMemcpyDeviceToHost, c->stream), "cutout D2H");
    std::vector<int64_t> ct(c->d.Tc);
    LPF_HIP(c, hipMemcpyAsync(ct.data(), c->buf.cache_t, c->d.Tc * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream),
            "cutout D2H");
    LPF_HIP(c, hipStreamSynchronize(c->stream), "cutout sync");
    if (have)
        for (int k = 0; k < n_steps; ++k) {
            const int64_t tau = t_first + k;
            have[k] = (c->n_frames > 0 && ct[pmod(tau, c->d.Tc)] == tau) ? 1 : 0;
        }
    return LPF_OK;
}

// ---- checkpoint / resume ----------------------------------------------------

namespace {

constexpr char kCkptMagic[8] = {'L', 'P', 'F', 'C', 'K', 'P', 'T', '1'};

// Fixed part of a checkpoint: the configuration values that fix the state's
// layout and meaning, and the host-side step bookkeeping.
struct CkptHeader {
    char magic[8];
    int32_t B, H, W, k, Tc, max_sources, peak_cap, kernel, clip_iters, peak_halfwidth, flux_halfwidth;
    int32_t monitor_steps, backfill_steps, qc_warmup, pipeline_ingest, filter_precision, masked, n_regions;
    float kappa, bg_sigma, dup_radius, assoc_radius, qc_band_z, qc_rms_z, qc_rms_floor, qc_pixel_zeta;
    int32_t grid_rows[kMaxB];
    int64_t t_last, t_start, n_frames;
    int32_t phase, pad;
};

CkptHeader ckpt_header(const lpf_ctx* c, int n_regions) {
    CkptHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kCkptMagic, sizeof(kCkptMagic));
    const lpf_config& f = c->cfg;
    h.B = f.B; h.H = f.H; h.W = f.W; h.k = c->d.k; h.Tc = c->d.Tc; h.max_sources = f.max_sources;
    h.peak_cap = f.peak_cap; h.kernel = f.kernel; h.clip_iters = f.clip_iters; h.peak_halfwidth = f.peak_halfwidth;
    h.flux_halfwidth = f.flux_halfwidth; h.monitor_steps = f.monitor_steps; h.backfill_steps = f.backfill_steps;
    h.qc_warmup = f.qc_warmup; h.pipeline_ingest = f.pipeline_ingest; h.filter_precision = f.filter_precision;
    h.masked = c->d.masked ? 1 : 0; h.n_regions = n_regions;
    h.kappa = f.kappa; h.bg_sigma = f.bg_sigma; h.dup_radius = f.dup_radius; h.assoc_radius = f.assoc_radius;
    h.qc_band_z = f.qc_band_z; h.qc_rms_z = f.qc_rms_z; h.qc_rms_floor = f.qc_rms_floor;
    h.qc_pixel_zeta = f.qc_pixel_zeta;
    for (int b = 0; b < kMaxB; ++b) h.grid_rows[b] = b < f.B ? c->grid_rows[b] : 0;
    h.t_last = c->t_last; h.t_start = c->t_start; h.n_frames = c->n_frames; h.phase = c->phase;
    return h;
}

struct Region {
    void* p;
    size_t bytes;
};

// Device state carried from one step to the next (D4-D7 and what a call
// after the last step may still read): image cache and its stamps, running
// QC statistics, sky mask, source table, free list, the last step's lists,
// counters, events and peaks, and the dynamic-spectrum rings.  Per-step
// scratch (filter planes, partials, candidate lists, catalogue scratch) is
// not part of it.
std::vector<Region> state_regions(lpf_ctx* c) {
    const DevBufs& b = c->buf;
    const size_t S = (size_t)c->cfg.max_sources, plane = c->d.plane, Tc = (size_t)c->d.Tc;
    const size_t B = (size_t)c->cfg.B;
    return {
        {b.cache, Tc * plane * sizeof(float)},
        {b.cache_t, Tc * sizeof(int64_t)},
        {b.cache_rej, Tc * sizeof(uint32_t)},
        {b.wf_mean, 2 * plane * sizeof(float)},
        {b.wf_m2, 2 * plane * sizeof(float)},
        {b.wf_n, kMaxB * sizeof(int32_t)},
        {b.wf_cur, kMaxB * sizeof(int32_t)},
        {b.mask, c->d.HW},
        {b.bandstats, 6 * kMaxB * sizeof(double)},
        {b.free_list, S * sizeof(int32_t)},
        {b.src_id, S * sizeof(int32_t)},
        {b.src_row, S * sizeof(int32_t)},
        {b.src_col, S * sizeof(int32_t)},
        {b.src_state, S * sizeof(int32_t)},
        {b.src_tfirst, S * sizeof(int64_t)},
        {b.src_tlast, S * sizeof(int64_t)},
        {b.src_tend, S * sizeof(int64_t)},
        {b.src_new, S * sizeof(int32_t)},
        {b.list_measured, S * sizeof(int2)},
        {b.list_new, S * sizeof(int2)},
        {b.list_ended, S * sizeof(int32_t)},
        {b.ring, S * B * kRing * sizeof(float)},
        {b.ring_t, S * kRing * sizeof(int64_t)},
        {b.ring_v, S * kRing * sizeof(uint32_t)},
        {b.status, sizeof(DevStatus)},
        {b.events, 2 * S * sizeof(lpf_source)},
        {b.peak_sorted, B * (size_t)c->cfg.peak_cap * sizeof(PeakRec)},
    };
}

size_t ckpt_bytes(lpf_ctx* c) {
    size_t n = sizeof(CkptHeader);
    for (const Region& r : state_regions(c)) n += sizeof(uint64_t) + r.bytes;
    return n;
}

}  // namespace

int lpf_checkpoint_size(lpf_ctx* c, size_t* bytes) {
    LPF_CHECK_CTX(c);
    if (!bytes) return fail(c, LPF_EINVAL, "null size");
    *bytes = ckpt_bytes(c);
    return LPF_OK;
}

int lpf_checkpoint_save(lpf_ctx* c, void* host, size_t bytes) {
    LPF_CHECK_CTX(c);
    if (!host) return fail(c, LPF_EINVAL, "null buffer");
    if (c->phase == 1 || c->phase == 2) return fail(c, LPF_ESTATE, "checkpoint between steps only (after extract_flux)");
    if (bytes < ckpt_bytes(c)) return fail(c, LPF_ENOMEM, "checkpoint buffer too small");
    LPF_HIP(c, sync_all(c), "checkpoint sync");
    const std::vector<Region> regs = state_regions(c);
    const CkptHeader h = ckpt_header(c, (int)regs.size());
    char* p = static_cast<char*>(host);
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    for (const Region& r : regs) {
        const uint64_t n = r.bytes;
        std::memcpy(p, &n, sizeof(n));
        p += sizeof(n);
        LPF_HIP(c, hipMemcpy(p, r.p, r.bytes, hipMemcpyDeviceToHost), "checkpoint D2H");
        p += r.bytes;
    }
    return LPF_OK;
}

int lpf_checkpoint_load(lpf_ctx* c, const void* host, size_t bytes) {
    LPF_CHECK_CTX(c);
    if (!host) return fail(c, LPF_EINVAL, "null buffer");
    if (c->n_frames != 0 || c->phase != 0) return fail(c, LPF_ESTATE, "load into a context that has taken no step");
    if (bytes < sizeof(CkptHeader)) return fail(c, LPF_EINVAL, "not a checkpoint");
    CkptHeader h;
    std::memcpy(&h, host, sizeof(h));
    const std::vector<Region> regs = state_regions(c);
    CkptHeader mine = ckpt_header(c, (int)regs.size());
    if (std::memcmp(h.magic, kCkptMagic, sizeof(kCkptMagic)) != 0) return fail(c, LPF_EINVAL, "not a checkpoint");
    // everything but the step bookkeeping must match this context
    mine.t_last = h.t_last;
    mine.t_start = h.t_start;
    mine.n_frames = h.n_frames;
    mine.phase = h.phase;
    if (std::memcmp(&h, &mine, sizeof(h)) != 0)
        return fail(c, LPF_EINVAL, "checkpoint of a different configuration");
    if (bytes < ckpt_bytes(c)) return fail(c, LPF_EINVAL, "checkpoint truncated");
    const char* p = static_cast<const char*>(host) + sizeof(h);
    LPF_HIP(c, sync_all(c), "checkpoint sync");
    // the sky mask is part of the configuration: it must equal this context's
    std::vector<uint8_t> cur(c->d.HW);
    for (const Region& r : regs) {
        uint64_t n = 0;
        std::memcpy(&n, p, sizeof(n));
        p += sizeof(n);
        if (n != r.bytes) return fail(c, LPF_EINVAL, "checkpoint region size mismatch");
        if (r.p == c->buf.mask) {
            LPF_HIP(c, hipMemcpy(cur.data(), r.p, r.bytes, hipMemcpyDeviceToHost), "mask D2H");
            if (std::memcmp(cur.data(), p, r.bytes) != 0) return fail(c, LPF_EINVAL, "checkpoint of a different sky mask");
        }
        p += r.bytes;
    }
    p = static_cast<const char*>(host) + sizeof(h);
    for (const Region& r : regs) {
        p += sizeof(uint64_t);
        LPF_HIP(c, hipMemcpy(r.p, p, r.bytes, hipMemcpyHostToDevice), "checkpoint H2D");
        p += r.bytes;
    }
    c->t_last = h.t_last;
    c->t_start = h.t_start;
    c->n_frames = h.n_frames;
    c->phase = h.phase;
    c->host_n_ended = -1;
    c->filt_recorded = false;
    c->qc_pending = false;
    return LPF_OK;
}

int lpf_status(lpf_ctx* c, lpf_status_t* out) {
    LPF_CHECK_CTX(c);
    if (!out) return LPF_EINVAL;
    DevStatus st;
    LPF_HIP(c, sync_all(c), "status sync");
    LPF_HIP(c, hipMemcpyAsync(&st, c->buf.status, sizeof(st), hipMemcpyDeviceToHost, c->stream), "status D2H");
    LPF_HIP(c, hipStreamSynchronize(c->stream), "status sync");
    out->t = c->t_last;
    out->rejected_bands = st.rejected;
    out->overflow_bands = st.overflow_bands;
    out->n_peaks = st.n_peaks;
    out->n_kept = st.n_kept;
    out->n_new = st.n_new;
    out->n_ended = st.n_ended;
    out->n_measured = st.n_measured;
    out->n_dropped = st.n_dropped;
    out->n_live = st.n_live;
    return LPF_OK;
}

int lpf_read_spectrum(lpf_ctx* c, int32_t id, float* out, uint8_t* valid, int64_t* t_last) {
    LPF_CHECK_CTX(c);
    if (!out) return LPF_EINVAL;
    const int S = c->cfg.max_sources, B = c->cfg.B;
    std::vector<int32_t> ids(S), state(S);
    LPF_HIP(c, sync_all(c), "spectrum sync");
    LPF_HIP(c, hipMemcpy(ids.data(), c->buf.src_id, S * sizeof(int32_t), hipMemcpyDeviceToHost), "ids D2H");
    LPF_HIP(c, hipMemcpy(state.data(), c->buf.src_state, S * sizeof(int32_t), hipMemcpyDeviceToHost), "state D2H");
    int slot = -1;
    for (int s = 0; s < S; ++s)
        if (state[s] != kSrcFree && ids[s] == id) {
            slot = s;
            break;
        }
    if (slot < 0) return fail(c, LPF_EINVAL, "source id not held");
    int64_t tend = c->t_last;
    if (state[slot] == kSrcEnded)
        LPF_HIP(c, hipMemcpy(&tend, c->buf.src_tend + slot, sizeof(int64_t), hipMemcpyDeviceToHost), "tend D2H");
    std::vector<float> ring((size_t)B * kRing);
    std::vector<int64_t> rt(kRing);
    std::vector<uint32_t> rv(kRing);
    LPF_HIP(c, hipMemcpy(ring.data(), c->buf.ring + (size_t)slot * B * kRing, ring.size() * sizeof(float),
                         hipMemcpyDeviceToHost), "ring D2H");
    LPF_HIP(c, hipMemcpy(rt.data(), c->buf.ring_t + (size_t)slot * kRing, kRing * sizeof(int64_t),
                         hipMemcpyDeviceToHost), "ring_t D2H");
    LPF_HIP(c, hipMemcpy(rv.data(), c->buf.ring_v + (size_t)slot * kRing, kRing * sizeof(uint32_t),
                         hipMemcpyDeviceToHost), "ring_v D2H");
    for (int col = 0; col < kRing; ++col) {
        const int64_t tau = tend - (kRing - 1) + col;
        const int ri = pmod(tau, kRing);
        for (int b = 0; b < B; ++b) {
            const bool ok = rt[ri] == tau && ((rv[ri] >> b) & 1u);
            out[(size_t)b * kRing + col] = ok ? ring[(size_t)b * kRing + ri] : 0.0f;
            if (valid) valid[(size_t)b * kRing + col] = ok ? 1 : 0;
        }
    }
    if (t_last) *t_last = tend;
    return LPF_OK;
}

int lpf_debug_read(lpf_ctx* c, int32_t what, void* host, size_t bytes) {
    LPF_CHECK_CTX(c);
    if (!host) return LPF_EINVAL;
    const size_t plane = c->d.plane;
    const void* src = nullptr;
    size_t need = 0;
    std::vector<int32_t> cur(kMaxB);
    LPF_HIP(c, sync_all(c), "debug sync");
    switch (what) {
        case LPF_DBG_BANDSTATS: src = c->buf.bandstats; need = (size_t)c->cfg.B * 6 * sizeof(double); break;
        case LPF_DBG_WELFORD_N: src = c->buf.wf_n; need = (size_t)c->cfg.B * sizeof(int32_t); break;
        case LPF_DBG_CENTRE: src = c->buf.centre; need = plane * sizeof(float); break;
        case LPF_DBG_SPREAD:
            if (!c->buf.spread) return fail(c, LPF_EINVAL, "spread plane not kept (debug_planes = 0)");
            src = c->buf.spread; need = plane * sizeof(float); break;
        case LPF_DBG_CLIPMASK:
            if (!c->buf.clip) return fail(c, LPF_EINVAL, "clip plane not kept");
            src = c->buf.clip + (size_t)(c->cfg.clip_iters & 1) * plane; need = plane; break;
        case LPF_DBG_CACHE:
            src = c->buf.cache + (size_t)pmod(c->t_last, c->d.Tc) * plane; need = plane * sizeof(float); break;
        case LPF_DBG_PREFILTERED:
            if (!c->buf.pre) return fail(c, LPF_EINVAL, "no PSF pre-filter (psf_sigma = 0)");
            src = c->buf.pre; need = plane * sizeof(float); break;
        case LPF_DBG_PEAKS:
        case LPF_DBG_EVENTS: {
            DevStatus st;
            LPF_HIP(c, hipMemcpy(&st, c->buf.status, sizeof(st), hipMemcpyDeviceToHost), "status D2H");
            if (what == LPF_DBG_PEAKS) {
                src = c->buf.peak_sorted;
                need = (size_t)std::max(st.n_peaks, 0) * sizeof(lpf_peak);
            } else {
                src = c->buf.events;
                need = (size_t)std::max(st.n_new + st.n_ended, 0) * sizeof(lpf_source);
            }
            if (need == 0 && bytes == 0) return LPF_OK;
            break;
        }
        case LPF_DBG_WELFORD_MEAN:
        case LPF_DBG_WELFORD_M2: {
            need = plane * sizeof(float);
            if (bytes != need) return fail(c, LPF_EINVAL, "size mismatch");
            LPF_HIP(c, hipMemcpy(cur.data(), c->buf.wf_cur, kMaxB * sizeof(int32_t), hipMemcpyDeviceToHost), "cur");
            const float* base = what == LPF_DBG_WELFORD_MEAN ? c->buf.wf_mean : c->buf.wf_m2;
            for (int b = 0; b < c->cfg.B; ++b) {
                const float* p = base + (size_t)cur[b] * plane + (size_t)b * c->d.HW;
                LPF_HIP(c, hipMemcpy(static_cast<char*>(host) + (size_t)b * c->d.HW * sizeof(float), p,
                                     c->d.HW * sizeof(float), hipMemcpyDeviceToHost), "welford D2H");
            }
            return LPF_OK;
        }
        default: return fail(c, LPF_EINVAL, "unknown buffer");
    }
    if (bytes != need) return fail(c, LPF_EINVAL, "size mismatch");
    LPF_HIP(c, hipMemcpy(host, src, need, hipMemcpyDeviceToHost), "debug D2H");
    return LPF_OK;
}

int lpf_profile_enable(lpf_ctx* c, int32_t stages) {
    LPF_CHECK_CTX(c);
    if (stages < 0 || stages > LPF_PROFILE_ALL) return fail(c, LPF_EINVAL, "stage mask");
    if (stages && c->prof_pool.empty()) {
        c->prof_pool.resize(1 << 14);
        for (auto& e : c->prof_pool)   // timing only: no system-scope fence around the kernels timed
            LPF_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "event create");
    }
    c->prof_mask = (uint32_t)stages;
    return LPF_OK;
}

int lpf_profile_read(lpf_ctx* c, double* ms, int64_t* counts) {
    LPF_CHECK_CTX(c);
    LPF_HIP(c, sync_all(c), "profile sync");
    for (int i = 0; i < LPF_STAGE_COUNT; ++i) {
        if (ms) ms[i] = 0.0;
        if (counts) counts[i] = 0;
    }
    for (const auto& r : c->prof_recs) {
        float e = 0.0f;
        LPF_HIP(c, hipEventElapsedTime(&e, r.a, r.b), "event time");
        if (ms) ms[r.stage] += e;
        if (counts) counts[r.stage] += 1;
    }
    c->prof_recs.clear();
    c->prof_next = 0;
    return LPF_OK;
}

int lpf_sync(lpf_ctx* c) {
    LPF_CHECK_CTX(c);
    LPF_HIP(c, sync_all(c), "sync");
    return LPF_OK;
}

const char* lpf_last_error(const lpf_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t lpf_model_weights_bytes(void) { return model_blob_bytes(); }

int lpf_model_workspace_size(int32_t precision, int32_t max_batch, size_t* bytes) {
    if (!bytes) return LPF_EINVAL;
    return model_workspace_size(precision, max_batch, bytes);
}

int lpf_model_create(const void* weights, size_t bytes, int32_t precision, int32_t max_batch, void* ws,
                     size_t ws_bytes, void* stream, lpf_model** out) {
    return model_create(weights, bytes, precision, max_batch, ws, ws_bytes, static_cast<hipStream_t>(stream), out);
}

void lpf_model_destroy(lpf_model* m) { model_destroy(m); }

int lpf_infer_windows(const lpf_model* m, const float* windows, int32_t n, float* mu, float* L, void* stream) {
    if (!m || (n > 0 && (!windows || !mu || !L)) || n < 0) return LPF_EINVAL;
    if (n == 0) return LPF_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int mb = m->max_batch;
    // the model's buffers are used in order on its own stream, between two events
    if (hipEventRecord(m->ev_in, s) != hipSuccess) return LPF_EDEVICE;
    if (hipStreamWaitEvent(m->istream, m->ev_in, 0) != hipSuccess) return LPF_EDEVICE;
    for (int i = 0; i < n; i += mb) {
        const int cnt = std::min(mb, n - i);
        hipError_t e = cnn_forward(m, windows + (size_t)i * kGridRows * kRing, nullptr, cnt, mu + (size_t)i * 4,
                                   L + (size_t)i * 10, m->istream);
        if (e != hipSuccess) return LPF_EDEVICE;
    }
    if (hipEventRecord(m->ev_out, m->istream) != hipSuccess) return LPF_EDEVICE;
    if (hipStreamWaitEvent(s, m->ev_out, 0) != hipSuccess) return LPF_EDEVICE;
    return LPF_OK;
}

int lpf_infer_windows_static(const lpf_model* m, const float* windows, int32_t n, float* mu, float* L,
                             void* stream) {
    if (!m || n < 0 || (n > 0 && (!windows || !mu || !L))) return LPF_EINVAL;
    if (n > static_max_windows()) return LPF_EINVAL;
    if (n == 0) return LPF_OK;
    hipError_t e = cnn_forward_static(m, windows, n, mu, L, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LPF_OK : LPF_EDEVICE;
}

int lpf_infer_async(lpf_ctx* const* ctxs, int32_t n_ctx, lpf_model* m, int64_t* ticket) {
    if (!ctxs || n_ctx < 1 || !m || !ticket) return LPF_EINVAL;
    for (int i = 0; i < n_ctx; ++i) {
        LPF_CHECK_CTX(ctxs[i]);
        if (ctxs[i]->phase != 3) return fail(ctxs[i], LPF_ESTATE, "infer needs extract_flux first");
    }
    lpf_ctx* c0 = ctxs[0];
    const int slot = (int)(m->next_ticket % kInflight);
    if (m->slot_ticket[slot] >= 0) return fail(c0, LPF_EFULL, "too many inference tickets outstanding");
    hipStream_t s = m->istream;
    const CnnWork& w = m->work;
    int32_t* hdr = w.sblk[slot];
    int32_t* rows = hdr + 4;
    float* win = w.swin[slot];
    if (n_ctx == 1) {
        // one context: its stream gathers into this ticket's buffers and goes
        // on; only the network waits (on the model's stream).  A pipelined
        // context defers the launch to after its next step's centre pass, so
        // the network runs beside that step's spread pass and catalogue.
        lpf_ctx* c = c0;
        if (c->ing_stream) {
            const int rc = flush_pending(c, nullptr);   // a ticket gathered earlier, no detect since
            if (rc != LPF_OK) return rc;
            LPF_HIP(c, launch_gather_ended(c, 0, hdr, win, rows, m->max_batch, c->stream, true), "gather");
            c->pend_model = m;
            c->pend_slot = slot;
            m->pend_ctx[slot] = c;
        } else {
            LPF_HIP(c, launch_gather_ended(c, 0, hdr, win, rows, m->max_batch, c->stream, true), "gather");
            LPF_HIP(c, hipEventRecord(m->ev_gath[slot], c->stream), "event record");
            const int rc = launch_ticket(m, slot, m->ev_gath[slot], c);
            if (rc != LPF_OK) return rc;
        }
    } else {
        // several contexts: their streams hand over to the model's stream
        // (flux and rings of this step are final), which gathers them in
        // order; each may go on as soon as its rings have been read
        for (int i = 0; i < n_ctx; ++i) {
            lpf_ctx* c = ctxs[i];
            if (!c->ev_ready) LPF_HIP(c, hipEventCreateWithFlags(&c->ev_ready, kDevEvent), "event");
            LPF_HIP(c, hipEventRecord(c->ev_ready, c->stream), "event record");
            LPF_HIP(c0, hipStreamWaitEvent(s, c->ev_ready, 0), "event wait");
        }
        for (int i = 0; i < n_ctx; ++i)
            LPF_HIP(ctxs[i], launch_gather_ended(ctxs[i], i, hdr, win, rows, m->max_batch, s, i == 0), "gather");
        LPF_HIP(c0, hipEventRecord(m->ev_gathered, s), "event record");
        for (int i = 0; i < n_ctx; ++i)
            LPF_HIP(ctxs[i], hipStreamWaitEvent(ctxs[i]->stream, m->ev_gathered, 0), "event wait");
        const int rc = launch_ticket(m, slot, m->ev_gathered, c0);
        if (rc != LPF_OK) return rc;
    }
    m->slot_ticket[slot] = m->next_ticket;
    *ticket = m->next_ticket++;
    return LPF_OK;
}

int lpf_infer_collect(lpf_model* m, int64_t ticket, float* mu_out, float* L_out, int32_t* src_out, int32_t cap,
                      int32_t* n_out) {
    if (!m || !n_out || ticket < 0) return LPF_EINVAL;
    const int slot = (int)(ticket % kInflight);
    if (m->slot_ticket[slot] != ticket) return LPF_EINVAL;
    if (m->pend_ctx[slot]) {   // launch not issued yet (no detect since the gather)
        const int rc = flush_pending(m->pend_ctx[slot], nullptr);
        if (rc != LPF_OK) return rc;
    }
    if (hipEventSynchronize(m->ev_done[slot]) != hipSuccess) return LPF_EDEVICE;
    const char* blk = m->h_res[slot];
    const int32_t* hdr = reinterpret_cast<const int32_t*>(blk);
    const int taken = hdr[0], seen = hdr[1];
    const int maxb = m->max_batch;
    const int32_t* rows = hdr + 4;
    const float* hmu = reinterpret_cast<const float*>(rows + 2 * (size_t)maxb);
    const float* hL = hmu + 4 * (size_t)maxb;
    // rows in (context, id) order
    std::vector<int> perm(taken);
    for (int k = 0; k < taken; ++k) perm[k] = k;
    std::sort(perm.begin(), perm.end(), [&](int x, int y) {
        return rows[2 * x] != rows[2 * y] ? rows[2 * x] < rows[2 * y] : rows[2 * x + 1] < rows[2 * y + 1];
    });
    const int nw = std::min(taken, std::max(cap, 0));
    for (int i = 0; i < nw; ++i) {
        const int k = perm[i];
        if (mu_out) std::memcpy(mu_out + (size_t)i * 4, hmu + (size_t)k * 4, 4 * sizeof(float));
        if (L_out) std::memcpy(L_out + (size_t)i * 10, hL + (size_t)k * 10, 10 * sizeof(float));
        if (src_out) { src_out[2 * i] = rows[2 * k]; src_out[2 * i + 1] = rows[2 * k + 1]; }
    }
    *n_out = nw;
    m->slot_ticket[slot] = -1;
    return seen > taken ? LPF_EFULL : LPF_OK;
}

int lpf_infer(lpf_ctx* const* ctxs, int32_t n_ctx, const lpf_model* m, const int32_t* ids, int32_t n_ids,
              float* mu_out, float* L_out, int32_t* src_out, int32_t cap, int32_t* n_out) {
    if (!ctxs || n_ctx < 1 || !m || !n_out) return LPF_EINVAL;
    if (ids && (n_ctx != 1 || n_ids < 0)) return LPF_EINVAL;
    for (int i = 0; i < n_ctx; ++i) {
        LPF_CHECK_CTX(ctxs[i]);
        if (ctxs[i]->phase != 3) return fail(ctxs[i], LPF_ESTATE, "infer needs extract_flux first");
    }
    lpf_ctx* c0 = ctxs[0];
    lpf_model* mm = const_cast<lpf_model*>(m);   // result slots and tickets
    if (!ids) {
        // device-driven: counts stay on the device, one wait for the results
        int64_t ticket = -1;
        int rc = lpf_infer_async(ctxs, n_ctx, mm, &ticket);
        if (rc != LPF_OK) return rc;
        rc = lpf_infer_collect(mm, ticket, mu_out, L_out, src_out, cap, n_out);
        if (rc != LPF_EFULL) return rc;
        // more ended episodes than the model's batch: host-driven chunks below
    }
    hipStream_t s = m->istream;
    const int mb = model_max_batch(m);
    float* win = model_window_buffer(m);
    float* dmu = model_mu_buffer(m);
    float* dL = model_L_buffer(m);
    // Entries: per context a run of windows gathered on the device.  With
    // ids == NULL the ended list of each context (slot order) is used and the
    // rows are reordered by id on the host afterwards; its count and ids come
    // from the read-back of detect when that took place.
    struct Run { int ctx; int n; std::vector<int32_t> id; };
    std::vector<Run> runs;
    int N = 0;
    for (int ci = 0; ci < n_ctx; ++ci) {
        lpf_ctx* c = ctxs[ci];
        Run r{ci, 0, {}};
        if (!ids) {
            if (c->host_n_ended < 0) {
                DevStatus st;
                LPF_HIP(c, hipMemcpyAsync(&st, c->buf.status, sizeof(st), hipMemcpyDeviceToHost, c->stream),
                        "status");
                LPF_HIP(c, hipStreamSynchronize(c->stream), "infer sync");
                std::vector<lpf_source> ev(st.n_ended);
                if (st.n_ended > 0)
                    LPF_HIP(c, hipMemcpy(ev.data(), c->buf.events + st.n_new, st.n_ended * sizeof(lpf_source),
                                         hipMemcpyDeviceToHost), "events");
                c->host_ended_ids.resize(st.n_ended);
                for (int k = 0; k < st.n_ended; ++k) c->host_ended_ids[k] = ev[k].id;
                c->host_n_ended = st.n_ended;
            }
            r.n = c->host_n_ended;
            if (r.n == 0) continue;
            LPF_HIP(c, launch_ended_ends(c, c->buf.infer_slots, c->buf.infer_tend), "ended list");
            r.id = c->host_ended_ids;
        } else {
            const int S = c->cfg.max_sources;
            std::vector<int32_t> idv(S), state(S);
            std::vector<int64_t> tend(S);
            LPF_HIP(c, sync_all(c), "infer sync");
            LPF_HIP(c, hipMemcpy(idv.data(), c->buf.src_id, S * sizeof(int32_t), hipMemcpyDeviceToHost), "ids");
            LPF_HIP(c, hipMemcpy(state.data(), c->buf.src_state, S * sizeof(int32_t), hipMemcpyDeviceToHost), "state");
            LPF_HIP(c, hipMemcpy(tend.data(), c->buf.src_tend, S * sizeof(int64_t), hipMemcpyDeviceToHost), "tend");
            std::vector<int32_t> sl(n_ids);
            std::vector<int64_t> te(n_ids);
            for (int k = 0; k < n_ids; ++k) {
                int slot = -1;
                for (int q = 0; q < S; ++q)
                    if (state[q] != kSrcFree && idv[q] == ids[k]) { slot = q; break; }
                if (slot < 0) return fail(c, LPF_EINVAL, "source id not held");
                sl[k] = slot;
                te[k] = state[slot] == kSrcEnded ? tend[slot] : c->t_last;
            }
            if (n_ids > 0) {
                LPF_HIP(c, hipMemcpy(c->buf.infer_slots, sl.data(), n_ids * sizeof(int32_t), hipMemcpyHostToDevice), "slots H2D");
                LPF_HIP(c, hipMemcpy(c->buf.infer_tend, te.data(), n_ids * sizeof(int64_t), hipMemcpyHostToDevice), "tend H2D");
            }
            r.n = n_ids;
            r.id.assign(ids, ids + n_ids);
        }
        if (r.n > 0) {
            N += r.n;
            runs.push_back(std::move(r));
        }
    }
    // rows in (context, id) order for the ended episodes, caller order for ids
    std::vector<int> row_ctx, row_id, row_src;  // row_src: index in gathered order
    {
        int base = 0;
        for (const auto& r : runs) {
            std::vector<int> perm(r.n);
            for (int k = 0; k < r.n; ++k) perm[k] = k;
            if (!ids) std::sort(perm.begin(), perm.end(), [&](int x, int y) { return r.id[x] < r.id[y]; });
            for (int k : perm) {
                row_ctx.push_back(r.ctx);
                row_id.push_back(r.id[k]);
                row_src.push_back(base + k);
            }
            base += r.n;
        }
    }
    *n_out = std::min(N, cap);
    if (N == 0) return LPF_OK;
    float* hrow = model_host_rows(m, N);   // pinned: the copies below stay asynchronous
    if (!hrow) return fail(c0, LPF_ENOMEM, "pinned result staging");
    // the contexts' streams hand their lists and rings over to the model's stream
    for (const auto& r : runs) {
        lpf_ctx* c = ctxs[r.ctx];
        if (!c->ev_ready) LPF_HIP(c, hipEventCreateWithFlags(&c->ev_ready, kDevEvent), "event");
        LPF_HIP(c, hipEventRecord(c->ev_ready, c->stream), "event record");
        LPF_HIP(c0, hipStreamWaitEvent(s, c->ev_ready, 0), "event wait");
    }
    // process the gathered rows in chunks of the model's batch; one wait at the end
    int g = 0;  // gathered index of the chunk start
    size_t run_i = 0;
    int run_off = 0;
    while (g < N) {
        const int cnt = std::min(mb, N - g);
        int filled = 0;
        while (filled < cnt) {
            const Run& r = runs[run_i];
            const int take = std::min(cnt - filled, r.n - run_off);
            lpf_ctx* c = ctxs[r.ctx];
            LPF_HIP(c0, launch_windows_gather(c, take, c->buf.infer_slots + run_off, c->buf.infer_tend + run_off,
                                              win + (size_t)filled * kGridRows * kRing, s), "windows");
            filled += take;
            run_off += take;
            if (run_off == r.n) { ++run_i; run_off = 0; }
        }
        {
            StageTimer tm(c0, 6, s);
            LPF_HIP(c0, cnn_forward(m, win, nullptr, cnt, dmu, dL, s), "cnn");
        }
        LPF_HIP(c0, hipMemcpyAsync(hrow + (size_t)g * 4, dmu, cnt * 4 * sizeof(float), hipMemcpyDeviceToHost, s),
                "mu D2H");
        LPF_HIP(c0, hipMemcpyAsync(hrow + (size_t)N * 4 + (size_t)g * 10, dL, cnt * 10 * sizeof(float),
                                   hipMemcpyDeviceToHost, s), "L D2H");
        g += cnt;
    }
    LPF_HIP(c0, hipStreamSynchronize(s), "infer sync");
    const float* hmu = hrow;
    const float* hL = hrow + (size_t)N * 4;
    const int nw = *n_out;
    for (int i = 0; i < nw; ++i) {
        const int k = row_src[i];
        if (mu_out) std::memcpy(mu_out + (size_t)i * 4, hmu + (size_t)k * 4, 4 * sizeof(float));
        if (L_out) std::memcpy(L_out + (size_t)i * 10, hL + (size_t)k * 10, 10 * sizeof(float));
        if (src_out) { src_out[2 * i] = row_ctx[i]; src_out[2 * i + 1] = row_id[i]; }
    }
    return LPF_OK;
}

}  // extern "C"
