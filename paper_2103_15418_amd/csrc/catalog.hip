// Source association and monitoring (Sec. 2.2), one workgroup per step.
//
// Input: the per-band peak lists written by the detection pass.  Steps:
// -1. (strip filters) the local-maximum test of the above-threshold pixels
//     the filter listed, appending peaks to the band lists;
//  0. release records reported as ended at the previous step; end episodes
//     a gap in t carried past their last measured step (done in the pass
//     that lists the live sources, 4a, which needs nothing from 1-3);
//  1. order all peaks by (band, row, col) -> the step's peak list;
//  2. order them by (x descending, band, row, col) -> visiting order;
//  3. duplicate removal: a peak is kept unless an earlier-visited kept peak
//     lies within dup_radius (greedy, in visiting order);
//  4. association: each kept peak, in visiting order, takes the nearest live
//     source within assoc_radius not taken this step (ties: lower id); else
//     a new source opens at its pixel (ids count up) if capacity allows;
//  5. episodes with t - t_last_det == monitor_steps end at this step (still
//     measured now); lists of measured / new / ended sources for the flux
//     and inference kernels, events for the host.
// Work is parallel over the workgroup (sorting networks, candidate search,
// compaction); only the two greedy resolutions, which are sequential by
// definition, run on one lane over short neighbour lists.

#include "lpf_internal.h"

namespace lpf {
namespace {

constexpr int kCatThreads = 1024;
// LDS capacities of the catalogue workgroup (about 42 KB in all, so that it
// can start on a CU that other kernels' workgroups already occupy); larger
// steps use the global scratch of the context (mostly L2-resident).
constexpr int kLdsKeys = 2048;                                 // sort keys (16 KB)
constexpr int kLdsPeaks = (kLdsKeys * 2) / (kNbr + 1);          // neighbour lists that fit the key area
constexpr int kLdsLive = kLdsKeys;                              // live (slot, position) pairs in the key area
constexpr int kLdsPos = 2048;                                   // positions and flags of listed peaks
constexpr int kLdsSrc = 16384;                                  // table slots of the taken / seen bitmaps
constexpr int kLdsKept = 256;                                   // kept peaks with LDS candidate lists
constexpr int kRowIndexMin = 512;   // above this many peaks the duplicate search buckets them by row

struct CatArgs {
    int B, peak_cap, max_sources, n_mon;
    float r_dup2, r_assoc2;
    int64_t t;
    int32_t* peak_cnt;
    PeakRec* peak_raw;
    int32_t* changed;        // per-iteration changed flags, cleared for the next step
    int n_changed;
    int32_t* cand_cnt;        // [1] above-threshold pixel count of the peak test, cleared for the next step
    int H;                    // image rows (row buckets of the duplicate search)
    PeakRec* peak_sorted;
    int32_t* order;     // [kCatMaxPeaks] bij-rank by visiting position
    int32_t* nbr;       // [kCatMaxPeaks][kNbr + 1]
    int32_t* cand;      // [kCatMaxPeaks][kCand + 1]
    int32_t* kept;      // [kCatMaxPeaks] kept peaks (visiting positions) in visiting order
    int32_t* dec;       // [kCatMaxPeaks] association decisions (large steps)
    uint64_t* g_keys;   // [kCatMaxPeaks] sort keys (steps with more than kLdsKeys peaks)
    int32_t* g_pos;     // [kCatMaxPeaks] positions in visiting order (large steps)
    uint8_t* g_flag;    // [kCatMaxPeaks] duplicate-removal flags (large steps)
    int32_t* g_live;    // [max_sources] live slots of this step
    int32_t* g_lpos;    // [max_sources] their positions
    uint32_t* g_taken;  // [max_sources / 32] bitmaps (tables beyond kLdsSrc slots)
    uint32_t* g_seen;
    int32_t* g_rowoff;  // [H + 1] row buckets of the duplicate search (many peaks)
    int32_t* g_rowcur;  // [H]
    int32_t* g_rowidx;  // [kCatMaxPeaks]
    int32_t* g_lrowidx; // [max_sources] live entries by row (association search, many sources)
    int32_t* free_list; // [max_sources]
    int32_t* src_id;
    int32_t* src_row;
    int32_t* src_col;
    int32_t* src_state;
    int64_t* src_tfirst;
    int64_t* src_tlast;
    int64_t* src_tend;
    int32_t* src_new;
    int2* list_measured;     // (slot, row << 16 | col): the flux kernel reads one record
    int2* list_new;
    int32_t* list_ended;
    int64_t* ring_t;
    DevStatus* status;
    lpf_source* events;
};

__device__ inline uint32_t ordered(float x) {
    uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ void bitonic_sort(uint64_t* k, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = k[lo], b = k[hi];
                if ((a > b) == up) {
                    k[lo] = b;
                    k[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

__device__ inline uint64_t shfl_xor_u64(uint64_t x, int m) {
    const int lo = __shfl_xor((int)(uint32_t)x, m, 64);
    const int hi = __shfl_xor((int)(uint32_t)(x >> 32), m, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Ascending sort of n (a power of two) keys; every thread of the block calls
// it.  Up to 64 keys are sorted in the registers of wave 0 (shuffle network,
// no block barriers); larger lists use the block-wide network in LDS.
__device__ void sort_keys(uint64_t* k, int n) {
    if (n <= 64) {
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            uint64_t x = lane < n ? k[lane] : ~0ull;
            for (int size = 2; size <= 64; size <<= 1) {
                for (int stride = size >> 1; stride > 0; stride >>= 1) {
                    const uint64_t y = shfl_xor_u64(x, stride);
                    const bool up = (lane & size) == 0;
                    const bool lower = (lane & stride) == 0;
                    x = (lower == up) ? (x < y ? x : y) : (x < y ? y : x);
                }
            }
            if (lane < n) k[lane] = x;
        }
        __syncthreads();
    } else {
        bitonic_sort(k, n);
    }
}

// Exclusive block scan of one int per thread; returns the prefix, *total = sum.
__device__ int block_scan(int v, int* s_tmp, int* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < kCatThreads / 64; ++i) {
            int t = s_tmp[i];
            s_tmp[i] = acc;
            acc += t;
        }
        s_tmp[kCatThreads / 64] = acc;
    }
    __syncthreads();
    int res = s_tmp[w] + x - v;
    *total = s_tmp[kCatThreads / 64];
    __syncthreads();
    return res;
}

// Three exclusive block scans at once: the counts are packed 21 bits apart
// into one 64-bit value (each count and total is below 2^21), so the block
// pays one set of barriers.  o[k]: prefixes, tot[k]: totals.
__device__ void block_scan3(const int* v, uint64_t* s_tmp64, int* o, int* tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t p = (uint64_t)v[0] | ((uint64_t)v[1] << 21) | ((uint64_t)v[2] << 42);
    uint64_t x = p;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int lo = __shfl_up((int)(uint32_t)x, d, 64);
        const int hi = __shfl_up((int)(uint32_t)(x >> 32), d, 64);
        if (lane >= d) x += ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    }
    if (lane == 63) s_tmp64[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int i = 0; i < kCatThreads / 64; ++i) {
            const uint64_t t = s_tmp64[i];
            s_tmp64[i] = acc;
            acc += t;
        }
        s_tmp64[kCatThreads / 64] = acc;
    }
    __syncthreads();
    const uint64_t res = s_tmp64[w] + x - p, t = s_tmp64[kCatThreads / 64];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o[k] = (int)((res >> (21 * k)) & 0x1fffffull);
        tot[k] = (int)((t >> (21 * k)) & 0x1fffffull);
    }
}

// Eight consecutive table entries s0 .. s0 + 7 of one thread (fill past S):
// 16-byte loads when the group is whole, so a wave touches each cache line
// once per instruction pair instead of once per entry.
__device__ inline void load8(const int32_t* p, int s0, int S, int fill, int* out) {
    if (s0 + 8 <= S) {
        const int4 a = *reinterpret_cast<const int4*>(p + s0);
        const int4 b = *reinterpret_cast<const int4*>(p + s0 + 4);
        out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
        out[4] = b.x; out[5] = b.y; out[6] = b.z; out[7] = b.w;
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) out[i] = s0 + i < S ? p[s0 + i] : fill;
    }
}

__device__ inline void store8(int32_t* p, int s0, int S, const int* v) {
    if (s0 + 8 <= S) {
        *reinterpret_cast<int4*>(p + s0) = make_int4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<int4*>(p + s0 + 4) = make_int4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (s0 + i < S) p[s0 + i] = v[i];
    }
}

__device__ inline void load8(const int64_t* p, int s0, int S, int64_t fill, int64_t* out) {
    if (s0 + 8 <= S) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const longlong2 v = *reinterpret_cast<const longlong2*>(p + s0 + 2 * h);
            out[2 * h] = v.x;
            out[2 * h + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) out[i] = s0 + i < S ? p[s0 + i] : fill;
    }
}

__device__ inline int pack_pos(int i, int j) { return (i << 16) | j; }
__device__ inline int pos_i(int p) { return p >> 16; }
__device__ inline int pos_j(int p) { return p & 0xffff; }
__device__ inline float dist2(int a, int b) {
    const float di = (float)(pos_i(a) - pos_i(b)), dj = (float)(pos_j(a) - pos_j(b));
    return di * di + dj * dj;
}

// Deferred local-maximum test (Sec. 2.1.2) of the above-threshold pixels the
// strip and disk filters listed, over many workgroups: a pixel is a peak if
// no pixel of its window inside the image and the sky mask exceeds it.
// Peaks are appended to their band's list (per-band counts in device memory;
// a band over peak_cap is dropped whole by the catalogue, which also orders
// the lists).  For the 7 x 7 window eight lanes share a pixel, one window row
// each, so a wave tests eight pixels with seven loads a lane.
struct PeakTestArgs {
    const int2* cand;      // (pixel index | band << 24, S bits)
    const int32_t* cand_cnt;
    const float* X;        // detection image [B][H][W]
    const float* C;        // centre plane
    const uint8_t* M;
    int H, W, kp, peak_cap;
    int32_t* peak_cnt;     // [B]
    PeakRec* peak_raw;     // [B][peak_cap]
};

__device__ inline void append_peak(const PeakTestArgs& a, int b, int gy, int gx, float xv, float cv, float sv) {
    const int idx = atomicAdd(&a.peak_cnt[b], 1);
    if (idx >= a.peak_cap) return;
    PeakRec rec;
    rec.band = b;
    rec.row = gy;
    rec.col = gx;
    rec.x = xv;
    rec.c = cv;
    rec.s = sv;
    rec.sig = (xv - cv) / sqrtf(sv);
    a.peak_raw[(size_t)b * a.peak_cap + idx] = rec;
}

__device__ __forceinline__ void peak_test_blocks(const PeakTestArgs& a, int blk, int nblk) {
    const int ncand = *a.cand_cnt;
    const size_t HW = (size_t)a.H * a.W;
    const int tid = threadIdx.x;
    if (a.kp == 3) {
        const int g = (blk * (int)blockDim.x + tid) >> 3, r = tid & 7;
        const int per_round = nblk * (int)blockDim.x / 8;
        for (int base = 0; base < ncand; base += per_round) {   // uniform trip count
            const int n = base + g;
            const bool valid = n < ncand;
            bool fail = false;
            int b = 0, gy = 0, gx = 0;
            float xv = 0.0f, cv = 0.0f, sv = 1.0f;
            if (valid) {
                const int2 e = a.cand[n];
                b = e.x >> 24;
                const int pix = e.x & 0xffffff;
                const float* Xb = a.X + (size_t)b * HW;
                gy = pix / a.W;
                gx = pix % a.W;
                sv = __int_as_float(e.y);
                xv = Xb[pix];
                if (r == 0) cv = a.C[(size_t)b * HW + pix];
                const int yy = gy + r - 3;
                if (r < 7 && yy >= 0 && yy < a.H) {
                    float v[7];
                    bool in[7];
#pragma unroll
                    for (int dx = 0; dx < 7; ++dx) {
                        const int xx = gx + dx - 3;
                        const int xc = xx < 0 ? 0 : (xx >= a.W ? a.W - 1 : xx);
                        const size_t p = (size_t)yy * a.W + xc;
                        v[dx] = Xb[p];
                        in[dx] = xx >= 0 && xx < a.W && (a.M ? a.M[p] != 0 : true);
                    }
#pragma unroll
                    for (int dx = 0; dx < 7; ++dx) fail = fail || (in[dx] && v[dx] > xv);
                }
            }
            const uint64_t bal = __ballot(fail);
            const bool peak = valid && ((bal >> (tid & 56)) & 0xffull) == 0ull;
            if (peak && r == 0) append_peak(a, b, gy, gx, xv, cv, sv);
        }
    } else {
        for (int n = blk * (int)blockDim.x + tid; n < ncand; n += nblk * (int)blockDim.x) {
            const int2 e = a.cand[n];
            const int b = e.x >> 24, pix = e.x & 0xffffff;
            const size_t bo = (size_t)b * HW;
            const int gy = pix / a.W, gx = pix % a.W;
            const float xv = a.X[bo + pix];
            if (window_max(a.X + bo, a.M, a.H, a.W, a.kp, gy, gx, xv))
                append_peak(a, b, gy, gx, xv, a.C[bo + pix], __int_as_float(e.y));
        }
    }
}

__global__ __launch_bounds__(256) void k_peak_test(PeakTestArgs a) { peak_test_blocks(a, blockIdx.x, gridDim.x); }

__global__ __launch_bounds__(256) void k_peak_test_group(Grouped<PeakTestArgs> g) {
    const int i = group_of(g.gi, blockIdx.x);
    peak_test_blocks(g.a[i], blockIdx.x - g.gi.start[i], g.gi.start[i + 1] - g.gi.start[i]);
}

// Counting sort of n items by the image row of their packed positions:
// rowoff[r] .. rowoff[r + 1] index the items of row r in idx (the order
// inside a row is that of the atomic cursor, which no result depends on).
// All threads of the workgroup call it; it ends with a barrier.
__device__ void bucket_rows(int n, const int32_t* pos, int32_t* rowoff, int32_t* rowcur, int32_t* idx, int H,
                            int* s_tmp) {
    const int tid = threadIdx.x;
    for (int r = tid; r <= H; r += kCatThreads) rowoff[r] = 0;
    __syncthreads();
    for (int q = tid; q < n; q += kCatThreads) atomicAdd(&rowoff[pos_i(pos[q])], 1);
    __syncthreads();
    {
        const int per = (H + kCatThreads - 1) / kCatThreads;
        const int r0 = tid * per, r1 = min(H, r0 + per);
        int sum = 0;
        for (int r = r0; r < r1; ++r) sum += rowoff[r];
        int tot;
        int acc = block_scan(sum, s_tmp, &tot);
        for (int r = r0; r < r1; ++r) {
            const int c = rowoff[r];
            rowoff[r] = acc;
            rowcur[r] = acc;
            acc += c;
        }
        if (tid == 0) rowoff[H] = tot;
    }
    __syncthreads();
    for (int q = tid; q < n; q += kCatThreads) idx[atomicAdd(&rowcur[pos_i(pos[q])], 1)] = q;
    __syncthreads();
}

__device__ __forceinline__ void catalog_body(const CatArgs& a) {
    __shared__ uint64_t s_keys[kLdsKeys];            // 16 KB: sort keys / neighbour lists / live lists
    __shared__ int32_t s_posl[kLdsPos];              //  8 KB: positions in visiting order
    __shared__ uint8_t s_flagl[kLdsPos];             //  2 KB: kept flags
    __shared__ uint32_t s_takenl[kLdsSrc / 32];      //  2 KB: taken bitmap
    __shared__ uint32_t s_seenl[kLdsSrc / 32];       //  2 KB: slots named by some candidate list
    __shared__ int32_t s_cand[kLdsKept * (kCand + 1)];  //  9 KB: candidate lists
    __shared__ int32_t s_dec[kLdsKept];              //  1 KB: association decisions
    __shared__ int32_t s_kept[kLdsKept];             //  1 KB: kept peaks (visiting positions)
    __shared__ int32_t s_freel[kLdsKept];            //  1 KB: first free slots of the table
    __shared__ uint64_t s_wkey[(kCatThreads / 64) * kCand];  // per-wave candidate keys
    __shared__ int32_t s_wslot[(kCatThreads / 64) * kCand];
    __shared__ int s_off[kMaxB + 1];
    __shared__ int s_cnt[kMaxB];
    __shared__ int s_tmp[kCatThreads / 64 + 1];
    __shared__ uint64_t s_tmp64[kCatThreads / 64 + 1];
    __shared__ int s_P, s_K, s_nlive, s_held, s_nfree, s_nnew, s_drop, s_next;
    __shared__ uint32_t s_overflow;

    const int tid = threadIdx.x;
    const int S = a.max_sources;
    const int64_t t = a.t;

    // per-band peak counts, read in parallel (one dependent read per band
    // would serialise as many memory latencies); the step's detection
    // counters are cleared for the next step's filters (the peak test,
    // earlier on this stream, has read the candidate count)
    if (tid < a.B) {
        s_cnt[tid] = a.peak_cnt[tid];
        a.peak_cnt[tid] = 0;
    }
    for (int i = tid; i < a.n_changed; i += kCatThreads) a.changed[i] = 0;
    if (tid == 0) a.cand_cnt[0] = 0;
    if (tid == kCatThreads - 1) s_next = a.status->next_id;   // in the same round trip
    __syncthreads();

    if (tid == 0) {
        int off = 0;
        uint32_t ovf = 0;
        for (int b = 0; b < a.B; ++b) {
            const int n = s_cnt[b];
            s_off[b] = off;
            if (n > a.peak_cap) ovf |= 1u << b;
            else off += n;
        }
        s_off[a.B] = off;
        s_P = off;
        s_overflow = ovf;
    }
    __syncthreads();
    const int P = s_P;

    // ---- 1. (band, row, col) order
    int Ppad = 1;
    while (Ppad < P) Ppad <<= 1;
    uint64_t* keys = Ppad <= kLdsKeys ? s_keys : a.g_keys;
    int32_t* s_pos = P <= kLdsPos ? s_posl : a.g_pos;
    uint8_t* s_flag = P <= kLdsPos ? s_flagl : a.g_flag;
    uint32_t* s_taken = S <= kLdsSrc ? s_takenl : a.g_taken;
    uint32_t* s_seen = S <= kLdsSrc ? s_seenl : a.g_seen;
    for (int n = tid; n < Ppad; n += kCatThreads) keys[n] = ~0ull;
    __syncthreads();
    int32_t* s_npos = s_cand;
    const bool pos_lds = P <= kLdsKept * (kCand + 1);
    if (P <= kCatThreads) {
        // one peak per lane, held in registers: the sorted copy and the
        // visiting-order keys are written from them through the rank of each
        // lane's peak (LDS), with no second read of the raw records
        PeakRec rec{};
        if (tid < P) {
            int b = 0;
            while (tid >= s_off[b + 1]) ++b;
            rec = a.peak_raw[(size_t)b * a.peak_cap + (tid - s_off[b])];
            const uint32_t key = ((uint32_t)rec.band << 24) | ((uint32_t)rec.row << 12) | (uint32_t)rec.col;
            keys[tid] = ((uint64_t)key << 32) | (uint32_t)tid;
        }
        __syncthreads();
        if (P > 1) sort_keys(keys, Ppad);
        int32_t* s_rank = s_posl;   // free until the visiting order is written
        if (tid < P) s_rank[(int)(keys[tid] & 0xffffffffu)] = tid;
        __syncthreads();
        if (tid < P) {
            const int n = s_rank[tid];
            a.peak_sorted[n] = rec;
            keys[n] = ((uint64_t)(~ordered(rec.x)) << 32) | (uint32_t)n;
            if (pos_lds) s_npos[n] = pack_pos(rec.row, rec.col);
        }
        __syncthreads();
    } else {
        // one pass over all listed peaks (overflowed bands have empty ranges)
        for (int n = tid; n < P; n += kCatThreads) {
            int b = 0;
            while (n >= s_off[b + 1]) ++b;
            const int q = n - s_off[b];
            const PeakRec& r = a.peak_raw[(size_t)b * a.peak_cap + q];
            const uint32_t key = ((uint32_t)r.band << 24) | ((uint32_t)r.row << 12) | (uint32_t)r.col;
            keys[n] = ((uint64_t)key << 32) | (uint32_t)(b * a.peak_cap + q);
        }
        __syncthreads();
        if (P > 1) sort_keys(keys, Ppad);
        // copy in (band, row, col) order; the same lane writes the visiting-order
        // key of position n (x descending, then rank n); padding keys stay ~0.
        // Positions also go to LDS (the candidate-list area, free until phase 4b)
        // when they fit, so the visiting order needs no read of the copy.
        for (int n = tid; n < P; n += kCatThreads) {
            const uint32_t ref = (uint32_t)(keys[n] & 0xffffffffu);
            const PeakRec rec = a.peak_raw[ref];
            a.peak_sorted[n] = rec;
            keys[n] = ((uint64_t)(~ordered(rec.x)) << 32) | (uint32_t)n;
            if (pos_lds) s_npos[n] = pack_pos(rec.row, rec.col);
        }
        __syncthreads();
    }

    // ---- 2. visiting order: x descending, then (band, row, col) = rank
    if (P > 1) sort_keys(keys, Ppad);
    for (int q = tid; q < P; q += kCatThreads) {
        const int n = (int)(keys[q] & 0xffffffffu);
        a.order[q] = n;
        s_pos[q] = pos_lds ? s_npos[n] : pack_pos(a.peak_sorted[n].row, a.peak_sorted[n].col);
    }
    __syncthreads();

    // ---- 3. duplicate removal: a peak is kept unless an earlier-visited kept
    // peak lies within dup_radius.  Up to 64 peaks: wave 0 holds one peak per
    // lane, builds each lane's 64-bit mask of earlier neighbours from
    // positions read lane by lane, and resolves the greedy order with one
    // mask test per peak.  More peaks: neighbour lists, then the greedy pass
    // on one lane.
    if (P <= 64) {
        if (tid < 64) {
            const int q = tid;
            const int pq = q < P ? s_pos[q] : 0;
            uint64_t nbm = 0ull;
            for (int r = 0; r < P; ++r) {   // uniform
                const int pr = __builtin_amdgcn_readlane(pq, r);
                if (r < q && dist2(pq, pr) <= a.r_dup2) nbm |= 1ull << r;
            }
            const uint32_t nlo = (uint32_t)nbm, nhi = (uint32_t)(nbm >> 32);
            uint64_t kept = 0ull;
            for (int j = 0; j < P; ++j) {   // uniform: the greedy order
                const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)nhi, j) << 32) |
                                   (uint32_t)__builtin_amdgcn_readlane((int)nlo, j);
                if ((m & kept) == 0ull) kept |= 1ull << j;
            }
            if (q < P) s_flag[q] = (uint8_t)((kept >> q) & 1ull);
            if (q < P && ((kept >> q) & 1ull)) {   // kept list in visiting order
                const int k = __popcll(kept & ((1ull << q) - 1ull));
                a.kept[k] = q;
                s_kept[k] = q;   // P <= 64 <= kLdsKept
            }
            if (q == 0) s_K = __popcll(kept);
        }
        __syncthreads();
    } else {
        // nbr[q] = {count, up to kNbr earlier-visited peaks within dup_radius};
        // held in LDS (the sort-key area) for steps with at most kLdsPeaks peaks.
        int32_t* nbr = P <= kLdsPeaks ? reinterpret_cast<int32_t*>(s_keys) : a.nbr;
        if (P <= kRowIndexMin) {
            for (int q = tid; q < P; q += kCatThreads) {
                const int pq = s_pos[q];
                int32_t* nb = nbr + (size_t)q * (kNbr + 1);
                int cnt = 0;
                for (int r = 0; r < q; ++r) {
                    if (dist2(pq, s_pos[r]) <= a.r_dup2) {
                        if (cnt < kNbr) nb[1 + cnt] = r;
                        ++cnt;
                    }
                }
                nb[0] = cnt;
            }
        } else {
            // many peaks: bucket them by image row (counting sort of the
            // visiting indices), then each peak looks only at the rows within
            // dup_radius of its own
            int32_t* rowoff = a.g_rowoff;   // [H + 1] bucket starts
            const int H = a.H;
            bucket_rows(P, s_pos, rowoff, a.g_rowcur, a.g_rowidx, H, s_tmp);
            const int R = (int)floorf(sqrtf(a.r_dup2));
            for (int q = tid; q < P; q += kCatThreads) {
                const int pq = s_pos[q];
                const int i = pos_i(pq);
                int32_t* nb = nbr + (size_t)q * (kNbr + 1);
                int cnt = 0;
                for (int rr = max(0, i - R); rr <= min(H - 1, i + R); ++rr) {
                    for (int e = rowoff[rr]; e < rowoff[rr + 1]; ++e) {
                        const int r = a.g_rowidx[e];
                        if (r < q && dist2(pq, s_pos[r]) <= a.r_dup2) {
                            if (cnt < kNbr) nb[1 + cnt] = r;
                            ++cnt;
                        }
                    }
                }
                nb[0] = cnt;
            }
        }
        __syncthreads();
        // The greedy order resolved in parallel rounds: a peak without an
        // earlier neighbour is kept whatever the others do; a peak with a kept
        // earlier neighbour is dropped; a peak whose earlier neighbours are all
        // dropped is kept.  Each round decides every peak whose earlier
        // neighbours are decided, which is the decision of the greedy pass (the
        // rounds follow its dependency chains, as deep as a cluster of
        // duplicates is long).  s_flag: 1 kept, 0 dropped, 2 undecided.
        for (int q = tid; q < P; q += kCatThreads) s_flag[q] = nbr[(size_t)q * (kNbr + 1)] == 0 ? 1 : 2;
        __syncthreads();
        for (;;) {
            int open = 0;
            for (int q = tid; q < P; q += kCatThreads) {
                if (s_flag[q] != 2) continue;
                const int32_t* nb = nbr + (size_t)q * (kNbr + 1);
                const int cnt = nb[0];
                bool kept_nb = false, pending = false;
                if (cnt > kNbr) {   // long list: every earlier peak within the radius
                    for (int r = 0; r < q && !kept_nb; ++r) {
                        if (dist2(s_pos[q], s_pos[r]) > a.r_dup2) continue;
                        const int f = s_flag[r];
                        kept_nb = f == 1;
                        pending = pending || f == 2;
                    }
                } else {
                    for (int r = 0; r < cnt && !kept_nb; ++r) {
                        const int f = s_flag[nb[1 + r]];
                        kept_nb = f == 1;
                        pending = pending || f == 2;
                    }
                }
                // a flag changes once, from 2 to its final value, so a decision
                // read in the same round it was written is already the final one
                if (kept_nb) s_flag[q] = 0;
                else if (!pending) s_flag[q] = 1;
                else open = 1;
            }
            if (!__syncthreads_or(open)) break;
        }
        {
            const int per = (P + kCatThreads - 1) / kCatThreads;
            const int q0 = tid * per, q1 = min(P, q0 + per);
            int nk = 0;
            for (int q = q0; q < q1; ++q) nk += s_flag[q];
            int tot;
            (void)block_scan(nk, s_tmp, &tot);
            if (tid == 0) s_K = tot;
        }
        __syncthreads();
    }
    const int K = s_K;
    if (P > 64) {   // kept list in visiting order (parallel compaction)
        const int per = (P + kCatThreads - 1) / kCatThreads;
        const int q0 = tid * per, q1 = min(P, q0 + per);
        int nk = 0;
        for (int q = q0; q < q1; ++q) nk += s_flag[q];
        int tot;
        int ok = block_scan(nk, s_tmp, &tot);
        for (int q = q0; q < q1; ++q)
            if (s_flag[q]) {
                a.kept[ok] = q;
                if (ok < kLdsKept) s_kept[ok] = q;
                ++ok;
            }
    }
    __syncthreads();

    // ---- 0 + 4a. release the records reported as ended at the previous step
    // and end the episodes left over by a gap, then list the live sources
    // (compacted, slot order) and the free slots, in one pass over the table
    for (int w = tid; w < (S + 31) / 32; w += kCatThreads) {
        s_taken[w] = 0u;
        s_seen[w] = 0u;
    }
    // live (slot, position) pairs go to the key area in LDS when the table is
    // scanned in one round and they fit, else to the global scratch (copied
    // to the key area afterwards when they fit)
    int32_t* s_live = reinterpret_cast<int32_t*>(s_keys);
    int32_t* s_lpos = s_live + kLdsLive;
    {
        // rounds of 8 consecutive slots per thread: the loads (state, last
        // detection, position) are issued together and the scan keeps slot order
        int base_l = 0, base_f = 0, base_h = 0;
        for (int base = 0; base < S; base += 8 * kCatThreads) {
            const int s0 = base + tid * 8;
            int st[8], row[8], col[8];
            int64_t tdet[8];
            load8(a.src_state, s0, S, -1, st);
            load8(a.src_tlast, s0, S, (int64_t)0, tdet);
            load8(a.src_row, s0, S, 0, row);
            load8(a.src_col, s0, S, 0, col);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (st[i] == kSrcEnded) {
                    st[i] = kSrcFree;
                } else if (st[i] == kSrcLive && t - tdet[i] > a.n_mon) {
                    st[i] = kSrcEnded;
                    a.src_tend[s0 + i] = tdet[i] + a.n_mon;   // live => s0 + i < S
                }
            }
            const int zeros[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            store8(a.src_state, s0, S, st);
            store8(a.src_new, s0, S, zeros);
            int nl = 0, nf = 0, nh = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                nl += st[i] == kSrcLive;
                nf += st[i] == kSrcFree;
                nh += st[i] == kSrcLive || st[i] == kSrcEnded;
            }
            int cnt[3] = {nl, nf, nh}, pre[3], tot3[3];
            block_scan3(cnt, s_tmp64, pre, tot3);
            const int tl = tot3[0], tf = tot3[1], th = tot3[2];
            int ol = base_l + pre[0];
            int of = base_f + pre[1];
            // a table of one round whose live list fits the LDS writes it there only
            const bool to_lds = S <= 8 * kCatThreads && tl <= kLdsLive;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int sl = s0 + i;
                if (st[i] == kSrcLive) {
                    if (to_lds) {
                        s_live[ol] = sl;
                        s_lpos[ol] = pack_pos(row[i], col[i]);
                    } else {
                        a.g_live[ol] = sl;
                        a.g_lpos[ol] = pack_pos(row[i], col[i]);
                    }
                    ++ol;
                } else if (st[i] == kSrcFree) {
                    a.free_list[of] = sl;
                    if (of < kLdsKept) s_freel[of] = sl;
                    ++of;
                }
            }
            base_l += tl;
            base_f += tf;
            base_h += th;
        }
        if (tid == 0) {
            s_nlive = base_l;
            s_nfree = base_f;
            s_held = base_h;
        }
    }
    __syncthreads();
    const int L = s_nlive;
    const bool live_in_lds = L <= kLdsLive;
    if (live_in_lds && S > 8 * kCatThreads) {   // several rounds: copy from the global list
        for (int l = tid; l < L; l += kCatThreads) {
            s_live[l] = a.g_live[l];
            s_lpos[l] = a.g_lpos[l];
        }
        __syncthreads();
    }
    const int32_t* live = live_in_lds ? s_live : a.g_live;
    const int32_t* lpos = live_in_lds ? s_lpos : a.g_lpos;

    // ---- 4b. association candidates of each kept peak, sorted by (d^2, id).
    // cand[kq] = {count or -1 (too many / table not staged), up to kCand slots}.
    // One wave per kept peak scans the live list 64 sources at a time.
    int32_t* cand = K <= kLdsKept ? s_cand : a.cand;
    int32_t* dec = K <= kLdsKept ? s_dec : a.dec;
    // many live sources and kept peaks: bucket the live list by row, so each
    // peak looks only at the rows within assoc_radius of its own
    const bool lbucket = L > kRowIndexMin && K > 64;
    if (lbucket) bucket_rows(L, lpos, a.g_rowoff, a.g_rowcur, a.g_lrowidx, a.H, s_tmp);
    {
        const int wave = tid >> 6, lane = tid & 63;
        uint64_t* wkey = s_wkey + wave * kCand;
        int32_t* wslot = s_wslot + wave * kCand;
        const int R = (int)floorf(sqrtf(a.r_assoc2));
        for (int kq = wave; kq < K; kq += kCatThreads / 64) {
            int32_t* out = cand + (size_t)kq * (kCand + 1);
            const int pq = s_pos[K <= kLdsKept ? s_kept[kq] : a.kept[kq]];
            // the live entries to test: all of them, or the rows i - R .. i + R
            const int pi = pos_i(pq);
            const int rr0 = lbucket ? max(0, pi - R) : 0, rr1 = lbucket ? min(a.H - 1, pi + R) : 0;
            int cnt = 0;
            for (int rr = rr0; rr <= rr1 && cnt <= kCand; ++rr) {
                const int e0 = lbucket ? a.g_rowoff[rr] : 0, e1 = lbucket ? a.g_rowoff[rr + 1] : L;
                for (int l0 = e0; l0 < e1 && cnt <= kCand; l0 += 64) {
                    const int e = l0 + lane;
                    const int l = e < e1 ? (lbucket ? a.g_lrowidx[e] : e) : 0;
                    const int lp = e < e1 ? lpos[l] : 0;
                    const bool hit = e < e1 && dist2(pq, lp) <= a.r_assoc2;
                    const uint64_t bal = __ballot(hit);
                    const int nh = __popcll(bal);
                    if (cnt + nh > kCand) {
                        cnt = kCand + 1;
                        break;
                    }
                    if (hit) {
                        const int at = cnt + __popcll(bal & ((1ull << lane) - 1ull));
                        const int s = live[l];
                        const uint32_t d2 = (uint32_t)dist2(pq, lp);
                        wkey[at] = ((uint64_t)d2 << 32) | (uint32_t)a.src_id[s];
                        wslot[at] = s;
                    }
                    cnt += nh;
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                if (cnt > kCand) {
                    out[0] = -1;
                } else {
                    // insertion sort of <= kCand (d^2, id) keys
                    for (int i = 1; i < cnt; ++i) {
                        const uint64_t kk = wkey[i];
                        const int ss = wslot[i];
                        int j = i - 1;
                        while (j >= 0 && wkey[j] > kk) {
                            wkey[j + 1] = wkey[j];
                            wslot[j + 1] = wslot[j];
                            --j;
                        }
                        wkey[j + 1] = kk;
                        wslot[j + 1] = ss;
                    }
                    out[0] = cnt;
                    for (int m = 0; m < cnt; ++m) out[1 + m] = wslot[m];
                }
            }
        }
    }
    __syncthreads();

    // ---- 4c. resolution in visiting order: dec[kq] = matched slot (>= 0),
    // -1 - r for the r-th new source, or INT32_MIN for a peak dropped at
    // capacity.  When every candidate list is complete and no slot appears in
    // two lists, no peak can take another's candidate: each takes its first
    // one and new sources are numbered by a prefix count (parallel).
    // Otherwise one lane resolves greedily on LDS data.
    int conflict = 0;
    for (int kq = tid; kq < K; kq += kCatThreads) {
        const int32_t* cl = cand + (size_t)kq * (kCand + 1);
        if (cl[0] < 0) {
            conflict = 1;
            continue;
        }
        for (int m = 0; m < cl[0]; ++m) {
            const int sl = cl[1 + m];
            const uint32_t bit = 1u << (sl & 31);
            if (atomicOr(&s_seen[sl >> 5], bit) & bit) conflict = 1;
        }
    }
    conflict = __syncthreads_or(conflict);
    if (!conflict) {
        const int per = (K + kCatThreads - 1) / kCatThreads;
        const int q0 = tid * per, q1 = min(K, q0 + per);
        int nw = 0;
        for (int kq = q0; kq < q1; ++kq) nw += cand[(size_t)kq * (kCand + 1)] == 0;
        const int room = min(S - s_held, s_nfree);   // read before the scan's barriers (tid 0 updates s_held)
        int tot;
        int r = block_scan(nw, s_tmp, &tot);
        for (int kq = q0; kq < q1; ++kq) {
            const int32_t* cl = cand + (size_t)kq * (kCand + 1);
            if (cl[0] > 0) {
                dec[kq] = cl[1];
            } else {
                dec[kq] = r < room ? -1 - r : INT32_MIN;
                ++r;
            }
        }
        if (tid == 0) {
            const int made = min(tot, max(room, 0));
            s_nnew = made;
            s_drop = tot - made;
            s_held = s_held + made;
        }
    } else if (tid == 0) {
        int held = s_held, nnew = 0, drop = 0;
        for (int kq = 0; kq < K; ++kq) {
            const int32_t* cl = cand + (size_t)kq * (kCand + 1);
            int match = -1;
            if (cl[0] < 0) {
                // exact scan of the whole table (sources opened this step are taken)
                const int pq = s_pos[a.kept[kq]];
                float bd = 0.0f;
                int bid = 0;
                for (int s = 0; s < S; ++s) {
                    if (a.src_state[s] != kSrcLive || a.src_new[s]) continue;
                    if ((s_taken[s >> 5] >> (s & 31)) & 1u) continue;
                    const float d = dist2(pq, pack_pos(a.src_row[s], a.src_col[s]));
                    if (d > a.r_assoc2) continue;
                    const int id = a.src_id[s];
                    if (match < 0 || d < bd || (d == bd && id < bid)) {
                        match = s;
                        bd = d;
                        bid = id;
                    }
                }
            } else {
                for (int m = 0; m < cl[0]; ++m) {
                    const int s = cl[1 + m];
                    if (!((s_taken[s >> 5] >> (s & 31)) & 1u)) {
                        match = s;
                        break;
                    }
                }
            }
            if (match >= 0) {
                s_taken[match >> 5] |= 1u << (match & 31);
                dec[kq] = match;
            } else if (held >= S || nnew >= s_nfree) {
                ++drop;
                dec[kq] = INT32_MIN;
            } else {
                ++held;
                dec[kq] = -1 - nnew;
                ++nnew;
            }
        }
        s_nnew = nnew;
        s_drop = drop;
        s_held = held;
    }
    __syncthreads();
    // ---- 4d. apply the decisions (parallel)
    for (int kq = tid; kq < K; kq += kCatThreads) {
        const int dq = dec[kq];
        if (dq >= 0) {
            a.src_tlast[dq] = t;
        } else if (dq != INT32_MIN) {
            const int r = -1 - dq;
            const int s = r < kLdsKept ? s_freel[r] : a.free_list[r];
            const int pos = s_pos[K <= kLdsKept ? s_kept[kq] : a.kept[kq]];   // (row << 16) | col
            a.src_id[s] = s_next + r;
            a.src_row[s] = pos >> 16;
            a.src_col[s] = pos & 0xffff;
            a.src_state[s] = kSrcLive;
            a.src_tfirst[s] = t;
            a.src_tlast[s] = t;
            a.src_tend[s] = -1;
            a.src_new[s] = 1;
        }
    }
    __syncthreads();
    if (tid == 0) s_next += s_nnew;
    __syncthreads();

    // ---- 5. end of monitoring, lists, events (rounds of 8 slots per thread)
    {
        int base_m = 0, base_n = 0, base_e = 0;
        int tn_all = s_nnew;  // new events come first in the event list
        for (int base = 0; base < S; base += 8 * kCatThreads) {
            const int s0 = base + tid * 8;
            int st[8], nw[8];
            int64_t tl[8], te8[8];
            load8(a.src_state, s0, S, -1, st);
            load8(a.src_new, s0, S, 0, nw);
            load8(a.src_tlast, s0, S, (int64_t)0, tl);
            load8(a.src_tend, s0, S, (int64_t)0, te8);
            int nm = 0, nn = 0, ne = 0;
            uint32_t now_end = 0u;   // bit i: monitoring ends at this step
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (st[i] == kSrcLive) {
                    ++nm;
                    nn += nw[i] != 0;
                    if (t - tl[i] == a.n_mon) {
                        st[i] = kSrcEnded;
                        te8[i] = t;
                        now_end |= 1u << i;
                    }
                }
                ne += st[i] == kSrcEnded;
            }
            // scans first: their barriers then wait on no outstanding stores
            int cnt[3] = {nm, nn, ne}, pre[3], tot3[3];
            block_scan3(cnt, s_tmp64, pre, tot3);
            const int tm = tot3[0], tn = tot3[1], te = tot3[2];
            int om = base_m + pre[0];
            int on = base_n + pre[1];
            int oe = base_e + pre[2];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int sl = s0 + i;
                if (st[i] < 0) continue;
                if ((now_end >> i) & 1u) {
                    a.src_state[sl] = kSrcEnded;
                    a.src_tend[sl] = t;
                }
                if (nw[i]) {
                    longlong2* rt = reinterpret_cast<longlong2*>(a.ring_t + (size_t)sl * kRing);
                    for (int r = 0; r < kRing / 2; ++r) rt[r] = make_longlong2(INT64_MIN, INT64_MIN);
                }
                const bool measured = st[i] == kSrcLive || (st[i] == kSrcEnded && te8[i] == t);
                const bool event = nw[i] || st[i] == kSrcEnded;
                // positions only for the (few) held sources, in one round trip with the event fields
                const int row = measured || event ? a.src_row[sl] : 0;
                const int col = measured || event ? a.src_col[sl] : 0;
                const int pos = (row << 16) | col;
                if (measured) a.list_measured[om++] = make_int2(sl, pos);
                if (event) {
                    lpf_source ev;
                    ev.id = a.src_id[sl];
                    ev.row = row;
                    ev.col = col;
                    ev.t_first = a.src_tfirst[sl];
                    ev.t_last_det = tl[i];
                    ev.t_end = te8[i];
                    if (nw[i]) {
                        a.list_new[on] = make_int2(sl, pos);
                        ev.event = LPF_EVENT_NEW;
                        a.events[on++] = ev;
                    }
                    if (st[i] == kSrcEnded) {
                        a.list_ended[oe] = sl;
                        ev.event = LPF_EVENT_ENDED;
                        a.events[tn_all + oe] = ev;
                        ++oe;
                    }
                }
            }
            base_m += tm;
            base_n += tn;
            base_e += te;
        }
        const int tm = base_m, tn = base_n, te = base_e;
        if (tid == 0) {
            DevStatus* st = a.status;
            st->n_peaks = P;
            st->n_kept = K;
            st->n_new = tn;
            st->n_ended = te;
            st->n_measured = tm;
            st->n_dropped = s_drop;
            st->n_live = s_held;
            st->overflow_bands = s_overflow;
            st->next_id = s_next;
            st->cat_truncated = 0;
        }
    }
}

__global__ __launch_bounds__(kCatThreads) void k_catalog(CatArgs a) {
    // the catalogue's chain of short phases is the step's critical path: its
    // waves take issue priority over other kernels' waves sharing the CU
    __builtin_amdgcn_s_setprio(3);
    catalog_body(a);
}

// Grouped: workgroup i runs the catalogue step of context i.
__global__ __launch_bounds__(kCatThreads) void k_catalog_group(Grouped<CatArgs> g) {
    catalog_body(g.a[blockIdx.x]);
}

__global__ void k_table_init(int32_t* src_state, int S, int64_t* cache_t, uint32_t* cache_rej, int Tc,
                             DevStatus* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) src_state[i] = kSrcFree;
    if (i < Tc) {
        cache_t[i] = INT64_MIN;
        cache_rej[i] = 0u;
    }
    if (i == 0) {
        DevStatus z{};
        *status = z;
    }
}

}  // namespace

inline int pmod_host(int64_t a, int m) {
    const int64_t r = a % m;
    return (int)(r < 0 ? r + m : r);
}

CatArgs catalog_args(lpf_ctx* c, int64_t t) {
    CatArgs a;
    a.B = c->cfg.B;
    a.peak_cap = c->cfg.peak_cap;
    a.max_sources = c->cfg.max_sources;
    a.n_mon = c->cfg.monitor_steps;
    a.r_dup2 = c->cfg.dup_radius * c->cfg.dup_radius;
    a.r_assoc2 = c->cfg.assoc_radius * c->cfg.assoc_radius;
    a.t = t;
    a.peak_cnt = c->buf.peak_cnt;
    a.peak_raw = c->buf.peak_raw;
    a.changed = c->buf.changed;
    a.n_changed = (kMaxIters + 1) * c->cfg.B;
    a.peak_sorted = c->buf.peak_sorted;
    a.cand_cnt = c->buf.cand_cnt;
    a.H = c->cfg.H;
    a.order = c->buf.cat_order;
    a.nbr = c->buf.cat_nbr;
    a.cand = c->buf.cat_cand;
    a.kept = c->buf.cat_kept;
    a.dec = c->buf.cat_dec;
    a.g_keys = c->buf.cat_gkeys;
    a.g_pos = c->buf.cat_gpos;
    a.g_flag = c->buf.cat_gflag;
    a.g_live = c->buf.cat_live;
    a.g_lpos = c->buf.cat_lpos;
    a.g_taken = c->buf.cat_taken;
    a.g_seen = c->buf.cat_seen;
    a.g_rowoff = c->buf.cat_rowoff;
    a.g_rowcur = c->buf.cat_rowcur;
    a.g_rowidx = c->buf.cat_rowidx;
    a.g_lrowidx = c->buf.cat_lrowidx;
    a.free_list = c->buf.free_list;
    a.src_id = c->buf.src_id;
    a.src_row = c->buf.src_row;
    a.src_col = c->buf.src_col;
    a.src_state = c->buf.src_state;
    a.src_tfirst = c->buf.src_tfirst;
    a.src_tlast = c->buf.src_tlast;
    a.src_tend = c->buf.src_tend;
    a.src_new = c->buf.src_new;
    a.list_measured = c->buf.list_measured;
    a.list_new = c->buf.list_new;
    a.list_ended = c->buf.list_ended;
    a.ring_t = c->buf.ring_t;
    a.status = c->buf.status;
    a.events = c->buf.events;
    return a;
}

// The filters of one clip iteration on the strip or disk paths leave the
// local-maximum test to k_peak_test, launched before the catalogue.
bool peaks_deferred(const lpf_ctx* c) { return (c->d.strip || c->d.disk) && c->cfg.clip_iters == 1; }

constexpr int kPeakTestBlocks = 128;

PeakTestArgs peak_test_args(lpf_ctx* c, int64_t t) {
    PeakTestArgs a;
    a.cand = c->buf.cand;
    a.cand_cnt = c->buf.cand_cnt;
    a.X = c->d.pre ? c->buf.pre : c->buf.cache + (size_t)pmod_host(t, c->d.Tc) * c->d.plane;
    a.C = c->buf.centre;
    a.M = c->d.masked ? c->buf.mask : nullptr;
    a.H = c->cfg.H;
    a.W = c->cfg.W;
    a.kp = c->cfg.peak_halfwidth;
    a.peak_cap = c->cfg.peak_cap;
    a.peak_cnt = c->buf.peak_cnt;
    a.peak_raw = c->buf.peak_raw;
    return a;
}

hipError_t launch_catalog(lpf_ctx* c, int64_t t) {
    if (peaks_deferred(c))
        hipLaunchKernelGGL(k_peak_test, dim3(kPeakTestBlocks), dim3(256), 0, c->stream, peak_test_args(c, t));
    hipLaunchKernelGGL(k_catalog, dim3(1), dim3(kCatThreads), 0, c->stream, catalog_args(c, t));
    return hipGetLastError();
}

hipError_t launch_catalog_group(lpf_ctx* const* cs, const int64_t* ts, int n, hipStream_t s) {
    {
        static_assert(sizeof(Grouped<PeakTestArgs>) <= 4096, "grouped kernel arguments exceed 4 KiB");
        Grouped<PeakTestArgs> g{};
        int m = 0, total = 0;
        for (int i = 0; i < n; ++i) {
            if (!peaks_deferred(cs[i])) continue;
            g.a[m] = peak_test_args(cs[i], ts[i]);
            g.gi.start[m] = total;
            total += kPeakTestBlocks;
            ++m;
        }
        g.gi.n = m;
        g.gi.start[m] = total;
        if (m > 0) hipLaunchKernelGGL(k_peak_test_group, dim3(total), dim3(256), 0, s, g);
    }
    static_assert(sizeof(Grouped<CatArgs>) <= 4096, "grouped kernel arguments exceed 4 KiB");
    Grouped<CatArgs> g{};
    g.gi.n = n;
    for (int i = 0; i < n; ++i) {
        g.a[i] = catalog_args(cs[i], ts[i]);
        g.gi.start[i] = i;
    }
    g.gi.start[n] = n;
    hipLaunchKernelGGL(k_catalog_group, dim3(n), dim3(kCatThreads), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_table_init(lpf_ctx* c) {
    const int n = c->cfg.max_sources > c->d.Tc ? c->cfg.max_sources : c->d.Tc;
    hipLaunchKernelGGL(k_table_init, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->buf.src_state,
                       c->cfg.max_sources, c->buf.cache_t, c->buf.cache_rej, c->d.Tc, c->buf.status);
    return hipGetLastError();
}

}  // namespace lpf
