// Internal definitions shared by the HIP translation units of liblpf.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "lpf.h"

namespace lpf {

constexpr int kMaxB = 16;          // subbands (the network grid has 16 rows)
constexpr int kMaxK = 40;          // background kernel half-width
constexpr int kMaxPeakK = 8;       // max-filter half-width
constexpr int kMaxFluxK = 8;       // flux box half-width
constexpr int kRing = 64;          // dynamic-spectrum window (network input width)
constexpr int kGridRows = 16;      // network input rows
constexpr int kMaxIters = 16;      // sigma-clip iterations
constexpr int kCatMaxPeaks = 8192; // peaks entering association per step
constexpr int kMaxDim = 4096;      // rows / columns (positions pack into 12 bits)
constexpr int kMaxSources = 65536;
constexpr int kMaxCutoutHalf = 32; // image cutouts of candidates: (2 h + 1)^2 pixels, h <= 32

// Background filter tiles: 64 x 64 outputs per 256-thread workgroup.
constexpr int kTileW = 64;
constexpr int kTileH = 64;
constexpr int kFiltThreads = 256;

struct Taps {
    float g[2 * kMaxK + 1];
    int k;
};

struct PeakRec {  // identical layout to lpf_peak
    int32_t band, row, col;
    float x, c, s, sig;
};
static_assert(sizeof(PeakRec) == sizeof(lpf_peak), "peak layout");

enum SrcState : int32_t { kSrcFree = 0, kSrcLive = 1, kSrcEnded = 2 };

// Per-(band, ingest block) partial reductions.
struct BandPartial {
    double sx;
    double sxx;
    int32_t nonfinite;
    float zmax;
    int32_t pad[2];
};

// Device-side counters of the current step.
struct DevStatus {
    int32_t n_peaks;        // listed peaks (non-overflowed bands)
    int32_t n_kept;         // after duplicate removal
    int32_t n_new;
    int32_t n_ended;
    int32_t n_measured;
    int32_t n_dropped;      // capacity drops this step
    int32_t n_live;         // held records after the step
    uint32_t overflow_bands;
    uint32_t rejected;
    int32_t next_id;
    int32_t cat_truncated;  // peaks beyond kCatMaxPeaks (never with valid configs)
    int32_t pad[5];
};

// Device buffers carved from the caller's workspace.
struct DevBufs {
    float* cache;          // [Tc][B][H][W]
    int64_t* cache_t;      // [Tc]
    uint32_t* cache_rej;   // [Tc]
    float* wf_mean;        // [2][B][H][W]
    float* wf_m2;          // [2][B][H][W]
    int32_t* wf_n;         // [B]
    int32_t* wf_cur;       // [B]
    uint8_t* mask;         // [H][W]
    uint32_t* mask_bits;   // [H][mwords] packed sky mask
    float* inv_den;        // [H][W] 1 / (G * M), 0 where G * M = 0
    float* centre;         // [B][H][W]
    float* resid;          // [B][H][W] E = M r |r|, r = X - C: signed squared residual (strip kernels)
    float* spread;         // [B][H][W] (debug or iterations > 1)
    uint8_t* clip;         // [B][H][W] (debug or iterations > 1)
    float* den;            // [B][H][W] (iterations > 1)
    BandPartial* partials; // [B][nblk]
    double* bandstats;     // [B][6]
    int32_t* changed;      // [kMaxIters + 1][B]
    int32_t* peak_cnt;     // [B]
    int2* cand;            // [B][H*W] above-threshold pixels awaiting the peak test (strip kernels)
    int32_t* cand_cnt;     // [B]
    PeakRec* peak_raw;     // [B][peak_cap]
    PeakRec* peak_sorted;  // [B * peak_cap]
    // catalogue scratch
    int32_t* cat_dec;      // [kCatMaxPeaks] association decisions (large steps)
    int32_t* cat_order;    // [kCatMaxPeaks]
    int32_t* cat_kept;     // [kCatMaxPeaks]
    int32_t* cat_nbr;      // [kCatMaxPeaks][kNbr]
    int32_t* cat_cand;     // [kCatMaxPeaks][kCand]
    uint64_t* cat_gkeys;   // [kCatMaxPeaks] sort keys beyond the workgroup's LDS
    int32_t* cat_gpos;     // [kCatMaxPeaks]
    uint8_t* cat_gflag;    // [kCatMaxPeaks]
    int32_t* cat_live;     // [max_sources] live slots of the step
    int32_t* cat_lpos;     // [max_sources] their positions
    uint32_t* cat_taken;   // [max_sources / 32] bitmaps beyond the LDS ones
    uint32_t* cat_seen;
    int32_t* cat_rowoff;   // [H + 1] row buckets of the duplicate search
    int32_t* cat_rowcur;   // [H]
    int32_t* cat_rowidx;   // [kCatMaxPeaks]
    int32_t* cat_lrowidx;  // [max_sources] live sources by row
    int32_t* free_list;    // [max_sources]
    // source table
    int32_t* src_id;
    int32_t* src_row;
    int32_t* src_col;
    int32_t* src_state;
    int64_t* src_tfirst;
    int64_t* src_tlast;
    int64_t* src_tend;
    int32_t* src_new;      // 1 if opened this step
    int2* list_measured;     // [max_sources] (slot, row << 16 | col)
    int2* list_new;          // [max_sources] (slot, row << 16 | col)
    int32_t* list_ended;
    // rings
    float* ring;           // [S][B][64]
    int64_t* ring_t;       // [S][64]
    uint32_t* ring_v;      // [S][64]
    DevStatus* status;
    lpf_source* events;    // [2 * max_sources] staging for host copies
    int32_t* infer_slots;  // [max_sources] slots of an inference batch
    int64_t* infer_tend;   // [max_sources] their window ends
    float* cutout;         // [Tc][B][2 kMaxCutoutHalf + 1]^2 staging of lpf_read_cutouts
    float* pre;            // [B][H][W] PSF-correlated detection image (psf_sigma > 0)
    float* inv_den_psf;    // [H][W] 1 / (G_psf * M) (psf_sigma > 0)
};

struct Derived {
    int k;         // background half-width
    int Tc;        // image cache depth
    int nblk;      // ingest blocks per band
    size_t HW;
    size_t plane;  // B * H * W
    int mwords;    // 32-bit words per packed mask row
    bool masked;
    bool dyn;      // iterations > 1 or debug planes: materialise S / Y
    bool strip;    // strip kernels (W % 4 == 0, k in {15, 24, 36}): residual plane E
    bool disk;     // circular uniform kernel (disk.hip)
    bool pre;      // PSF pre-filter: detection runs on buf.pre
    int kpsf;      // its half-width
};

}  // namespace lpf

struct lpf_ctx {
    lpf_config cfg;
    int32_t grid_rows[lpf::kMaxB];
    lpf::Derived d;
    lpf::Taps taps;
    lpf::Taps taps_psf;   // PSF pre-filter taps (psf_sigma > 0)
    lpf::DevBufs buf;
    hipStream_t stream;
    int64_t t_last;
    int64_t t_start;
    int64_t n_frames;
    int phase;      // 0 fresh / after flux, 1 ingested, 2 detected, 3 measured
    bool poisoned;
    std::string err;
    // stage timing (lpf_profile_enable)
    uint32_t prof_mask = 0;   // stages timed (bit i = stage i)
    std::vector<hipEvent_t> prof_pool;
    size_t prof_next = 0;
    struct ProfRec { int stage; hipEvent_t a, b; };
    std::vector<ProfRec> prof_recs;
    // ended episodes of the last detect as read back by it (count -1: not read)
    int32_t host_n_ended = -1;
    std::vector<int32_t> host_ended_ids;   // list order (the order of the ended-slot list)
    hipEvent_t ev_ready = nullptr;         // cross-stream hand-off in pooled inference
    // pipelined ingest: ingest + QC on ing_stream, ordered after the previous
    // step's filters (ev_filt); the next detect waits for the QC (ev_qc)
    hipStream_t ing_stream = nullptr;
    hipEvent_t ev_filt = nullptr, ev_qc = nullptr;
    hipEvent_t ev_centre = nullptr;   // after this step's centre pass (deferred network launch)
    bool filt_recorded = false, qc_pending = false;
    // pipelined: a gathered inference ticket whose network launch waits for
    // this context's next centre pass (or its collect)
    lpf_model* pend_model = nullptr;
    int pend_slot = -1;
};

namespace lpf {

struct ModelLayout {
    // float offsets inside the weight area
    size_t w1, b1, w2, b2, w3, b3, w4, b4, f1, fb1, f2, fb2, total;
};

constexpr int kInflight = 4;   // asynchronous inference tickets outstanding per model

struct CnnWork {
    float* act_a;     // [maxb][16][64][64] (float32 network)
    float* act_b;
    void* act16_a;    // [maxb][16][64][64] (16-bit network)
    void* act16_b;
    void* w16;        // 16-bit weights: conv2..4 [9][Cout][Cin], fc1 [128][65536]
    float* part;      // [128][maxb_pad][128] fc1 split-K partials
    float* windows;   // [maxb][16][64]
    // result block, one contiguous device range (copied to the host in one piece):
    int32_t* hdr;     // [4]: windows taken, ended episodes seen
    int32_t* rows;    // [maxb][2]: (context index, source id)
    float* mu;        // [maxb][4]
    float* L;         // [maxb][10]
    size_t out_bytes; // bytes of the result block
    // per-ticket gather windows and result blocks (same layout as above) of
    // the asynchronous calls, so a batch can be gathered while the network
    // still reads the previous one
    float* swin[kInflight];
    int32_t* sblk[kInflight];
};

}  // namespace lpf

struct lpf_model {
    int precision;
    int max_batch;
    float alpha;
    float* wts;
    lpf::ModelLayout lay;
    lpf::CnnWork work;
    hipStream_t stream;            // the caller's stream (weight upload)
    hipStream_t istream = nullptr; // inference stream owned by the model
    hipEvent_t ev_gathered = nullptr, ev_in = nullptr, ev_out = nullptr;
    hipEvent_t ev_done[lpf::kInflight] = {};
    hipEvent_t ev_gath[lpf::kInflight] = {};   // per-ticket gather done (single-context calls)
    lpf_ctx* pend_ctx[lpf::kInflight] = {};    // context holding the ticket's deferred launch
    char* h_res[lpf::kInflight] = {};          // pinned result blocks
    int64_t slot_ticket[lpf::kInflight] = {-1, -1, -1, -1};
    int64_t next_ticket = 0;
    // pinned host staging for host-driven inference (grown on demand)
    mutable float* h_out = nullptr;
    mutable size_t h_cap = 0;   // rows
};

namespace lpf {

constexpr int kNbr = 16;   // stored higher-priority neighbours per peak
constexpr int kCand = 8;   // stored association candidates per kept peak

inline int xcd_count() { return 8; }

// Grouped launches (the batch calls): one kernel launch serves up to
// kGroupMax contexts; context i owns the flat workgroups [start[i],
// start[i+1]) and its arguments travel in the kernel-argument segment.
constexpr int kGroupMax = 8;
struct GroupIndex {
    int n;
    int start[kGroupMax + 1];
};
template <typename A>
struct Grouped {
    GroupIndex gi;
    A a[kGroupMax];
};
// Context of flat workgroup blk (wave-uniform).
__device__ inline int group_of(const GroupIndex& g, int blk) {
    int i = 0;
    while (i + 1 < g.n && blk >= g.start[i + 1]) ++i;
    return i;
}

// Local-maximum test of Sec. 2.1.2 at (y, x) of one band plane X: no pixel
// of the (2 KP + 1)^2 window inside the image and the sky mask M (null = all)
// exceeds xv, so ties are peaks.  Every window load is issued (from clamped,
// always valid addresses) before the comparisons.
template <int KP>
__device__ inline bool window_max_all(const float* X, const uint8_t* M, int H, int W, int y, int x, float xv) {
    constexpr int N = 2 * KP + 1;
    float v[N * N];
    bool in[N * N];
#pragma unroll
    for (int dy = 0; dy < N; ++dy) {
        const int yy = y + dy - KP;
        const bool rok = yy >= 0 && yy < H;
        const int yc = yy < 0 ? 0 : (yy >= H ? H - 1 : yy);
#pragma unroll
        for (int dx = 0; dx < N; ++dx) {
            const int xx = x + dx - KP;
            const int xc = xx < 0 ? 0 : (xx >= W ? W - 1 : xx);
            const size_t p = (size_t)yc * W + xc;
            v[dy * N + dx] = X[p];
            in[dy * N + dx] = rok && xx >= 0 && xx < W && (M ? M[p] != 0 : true);
        }
    }
    bool peak = true;
#pragma unroll
    for (int i = 0; i < N * N; ++i) peak = peak && !(in[i] && v[i] > xv);
    return peak;
}

// The same test for a run-time half-width kp.
__device__ inline bool window_max(const float* X, const uint8_t* M, int H, int W, int kp, int y, int x, float xv) {
    if (kp == 3) return window_max_all<3>(X, M, H, W, y, x, xv);
    for (int dy = -kp; dy <= kp; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= H) continue;
        for (int dx = -kp; dx <= kp; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= W) continue;
            const size_t p = (size_t)yy * W + xx;
            if (M && !M[p]) continue;
            if (X[p] > xv) return false;
        }
    }
    return true;
}

// Stage timer: records an event pair around the enclosed launches.
struct StageTimer {
    lpf_ctx* c;
    int stage;
    hipStream_t s;
    hipEvent_t b = nullptr;
    StageTimer(lpf_ctx* ctx, int st, hipStream_t on = nullptr) : c(ctx), stage(st), s(on ? on : ctx->stream) {
        if (!((c->prof_mask >> stage) & 1u) || c->prof_next + 2 > c->prof_pool.size()) return;
        hipEvent_t a = c->prof_pool[c->prof_next++];
        b = c->prof_pool[c->prof_next++];
        (void)hipEventRecord(a, s);
        c->prof_recs.push_back({stage, a, b});
    }
    ~StageTimer() {
        if (b) (void)hipEventRecord(b, s);
    }
};

// Launchers (defined in the .hip files); return hipError_t of the launch.
hipError_t launch_ingest(lpf_ctx* c, const float* src, bool copy, int slot, hipStream_t s);
hipError_t launch_qc_decide(lpf_ctx* c, int slot, int64_t t, hipStream_t s);
hipError_t launch_filters(lpf_ctx* c, int slot);
hipError_t launch_inv_den(lpf_ctx* c);
hipError_t launch_pack_mask(lpf_ctx* c);
hipError_t launch_catalog(lpf_ctx* c, int64_t t);
hipError_t launch_flux(lpf_ctx* c, int slot, int64_t t);
hipError_t launch_table_init(lpf_ctx* c);
hipError_t launch_disk_inv_den(lpf_ctx* c);
hipError_t launch_disk_filters(lpf_ctx* c, const float* X, const uint32_t* rej, hipStream_t s);
int disk_max_halfwidth();
hipError_t launch_prefilter(lpf_ctx* c, int slot);
hipError_t launch_cutouts(lpf_ctx* c, int row, int col, int half, int64_t t_first, int n_steps);
// grouped forms (n <= kGroupMax contexts on stream s)
hipError_t launch_ingest_group(lpf_ctx* const* cs, const float* const* srcs, const int* slots, int n, bool copy,
                               bool vec, hipStream_t s);
hipError_t launch_qc_decide_group(lpf_ctx* const* cs, const int* slots, const int64_t* ts, int n, hipStream_t s);
hipError_t launch_filters_group(lpf_ctx* const* cs, const int* slots, int n, hipStream_t s);
bool filters_groupable(const lpf_ctx* a, const lpf_ctx* b);
hipError_t launch_catalog_group(lpf_ctx* const* cs, const int64_t* ts, int n, hipStream_t s);
hipError_t launch_flux_group(lpf_ctx* const* cs, const int64_t* ts, int n, hipStream_t s);

}  // namespace lpf
