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
    float* spread;         // [B][H][W] (debug or iterations > 1)
    uint8_t* clip;         // [B][H][W] (debug or iterations > 1)
    float* den;            // [B][H][W] (iterations > 1)
    BandPartial* partials; // [B][nblk]
    double* bandstats;     // [B][6]
    int32_t* changed;      // [kMaxIters + 1][B]
    int32_t* peak_cnt;     // [B]
    PeakRec* peak_raw;     // [B][peak_cap]
    PeakRec* peak_sorted;  // [B * peak_cap]
    // catalogue scratch
    int32_t* cat_dec;      // [kCatMaxPeaks] association decisions (large steps)
    int32_t* cat_order;    // [kCatMaxPeaks]
    int32_t* cat_kept;     // [kCatMaxPeaks]
    int32_t* cat_nbr;      // [kCatMaxPeaks][kNbr]
    int32_t* cat_cand;     // [kCatMaxPeaks][kCand]
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
    int32_t* list_measured;  // [max_sources]
    int32_t* list_new;
    int32_t* list_ended;
    // rings
    float* ring;           // [S][B][64]
    int64_t* ring_t;       // [S][64]
    uint32_t* ring_v;      // [S][64]
    DevStatus* status;
    lpf_source* events;    // [2 * max_sources] staging for host copies
    float* windows;        // unused (network inputs live in the model workspace)
    int32_t* infer_slots;  // [max_sources] slots of an inference batch
    int64_t* infer_tend;   // [max_sources] their window ends
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
};

}  // namespace lpf

struct lpf_ctx {
    lpf_config cfg;
    int32_t grid_rows[lpf::kMaxB];
    lpf::Derived d;
    lpf::Taps taps;
    lpf::DevBufs buf;
    hipStream_t stream;
    int64_t t_last;
    int64_t t_start;
    int64_t n_frames;
    int phase;      // 0 fresh / after flux, 1 ingested, 2 detected, 3 measured
    bool poisoned;
    std::string err;
    // stage timing (lpf_profile_enable)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_next = 0;
    struct ProfRec { int stage; hipEvent_t a, b; };
    std::vector<ProfRec> prof_recs;
};

namespace lpf {

constexpr int kNbr = 16;   // stored higher-priority neighbours per peak
constexpr int kCand = 8;   // stored association candidates per kept peak

inline int xcd_count() { return 8; }

// Stage timer: records an event pair around the enclosed launches.
struct StageTimer {
    lpf_ctx* c;
    int stage;
    hipEvent_t b = nullptr;
    StageTimer(lpf_ctx* ctx, int st) : c(ctx), stage(st) {
        if (!c->prof_on || c->prof_next + 2 > c->prof_pool.size()) return;
        hipEvent_t a = c->prof_pool[c->prof_next++];
        b = c->prof_pool[c->prof_next++];
        (void)hipEventRecord(a, c->stream);
        c->prof_recs.push_back({stage, a, b});
    }
    ~StageTimer() {
        if (b) (void)hipEventRecord(b, c->stream);
    }
};

// Launchers (defined in the .hip files); return hipError_t of the launch.
hipError_t launch_ingest(lpf_ctx* c, const float* src, bool copy, int slot);
hipError_t launch_qc_decide(lpf_ctx* c, int slot, int64_t t);
hipError_t launch_detect_init(lpf_ctx* c);
hipError_t launch_filters(lpf_ctx* c, int slot);
hipError_t launch_inv_den(lpf_ctx* c);
hipError_t launch_pack_mask(lpf_ctx* c);
hipError_t launch_catalog(lpf_ctx* c, int64_t t);
hipError_t launch_flux(lpf_ctx* c, int slot, int64_t t);
hipError_t launch_table_init(lpf_ctx* c);

}  // namespace lpf
