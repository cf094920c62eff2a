// Flux measurement, backward fill and dynamic-spectrum windows (Sec. 2.2,
// Fig. 3).
//
// The flux of a source in a band is the maximum pixel value of the
// quality-controlled image in a (2k_f + 1)^2 box (clipped to the image)
// around the source's pixel; a band discarded by QC reads as zeros, so its
// flux is 0 and it is marked invalid.  Each measured source writes one value
// per band into its ring F[slot][band][tau mod 64] with the step tau in
// ring_t[slot][tau mod 64] and the valid-band bits in ring_v.  New sources
// are also measured on the cached steps [max(t - T_bf, t_start), t - 1].
// One lane per (source, band[, step]); the lists and their lengths come
// from the catalogue kernel in device memory, so grids are fixed-size and
// every lane runs a bounded grid-stride loop.

#include "lpf_internal.h"

namespace lpf {
namespace {

struct FluxArgs {
    const float* cache;       // [Tc][B][H][W]
    const int64_t* cache_t;   // [Tc]
    const uint32_t* cache_rej;
    int Tc, B, H, W, kf, T_bf;
    int bgw;                  // > 0: subtract the mean of the annulus this wide around the box
    int64_t t, t_start;
    size_t plane;
    const int2* list;         // measured sources (slot, row << 16 | col)
    const int32_t* count;     // their device count
    const int2* list_new;     // sources opened at this step (backward fill)
    const int32_t* count_new;
    int cap;                  // entries the lists can hold
    int flux_blocks;          // blocks [0, flux_blocks) measure, the rest fill backwards
    float* ring;
    int64_t* ring_t;
    uint32_t* ring_v;
};

__device__ inline int pmod(int64_t a, int m) {
    int64_t r = a % m;
    return (int)(r < 0 ? r + m : r);
}

__device__ inline float box_max(const float* img, int H, int W, int i, int j, int k) {
    const int r0 = i - k < 0 ? 0 : i - k, r1 = i + k >= H ? H - 1 : i + k;
    const int c0 = j - k < 0 ? 0 : j - k, c1 = j + k >= W ? W - 1 : j + k;
    float m = -INFINITY;
    for (int r = r0; r <= r1; ++r)
        for (int c = c0; c <= c1; ++c) m = fmaxf(m, img[(size_t)r * W + c]);
    return m;
}

// Box maximum with the half-width fixed at compile time: every load of the
// window (clamped addresses, always valid) is issued before the maxima, which
// are taken over the pixels inside the image in the same row-major order.
template <int KF>
__device__ inline float box_max_k(const float* img, int H, int W, int i, int j) {
    constexpr int N = 2 * KF + 1;
    float v[N * N];
    bool ok[N * N];
#pragma unroll
    for (int dr = 0; dr < N; ++dr) {
        const int r = i + dr - KF;
        const int rc = r < 0 ? 0 : (r >= H ? H - 1 : r);
#pragma unroll
        for (int dc = 0; dc < N; ++dc) {
            const int c = j + dc - KF;
            const int cc = c < 0 ? 0 : (c >= W ? W - 1 : c);
            v[dr * N + dc] = img[(size_t)rc * W + cc];
            ok[dr * N + dc] = r >= 0 && r < H && c >= 0 && c < W;
        }
    }
    float m = -INFINITY;
#pragma unroll
    for (int q = 0; q < N * N; ++q)
        if (ok[q]) m = fmaxf(m, v[q]);
    return m;
}

// Half-width 2 on rows of whole float4 (W % 4 == 0, W >= 8): two aligned
// 16-byte loads per row, starting at the multiple of 4 at or below j - 2
// (clamped to [0, W - 8]), hold the box's five columns; the maximum runs over
// the loaded pixels inside the box and the image, in the same row-major order
// as box_max_k<2>.
__device__ inline float box_max_2v(const float* img, int H, int W, int i, int j) {
    int a0 = (j - 2) & ~3;
    a0 = a0 < 0 ? 0 : (a0 > W - 8 ? W - 8 : a0);
    float v[5][8];
    bool rok[5];
#pragma unroll
    for (int dr = 0; dr < 5; ++dr) {
        const int r = i + dr - 2;
        const int rc = r < 0 ? 0 : (r >= H ? H - 1 : r);
        rok[dr] = r >= 0 && r < H;
        const float4* p = reinterpret_cast<const float4*>(img + (size_t)rc * W + a0);
        const float4 lo = p[0], hi = p[1];
        v[dr][0] = lo.x; v[dr][1] = lo.y; v[dr][2] = lo.z; v[dr][3] = lo.w;
        v[dr][4] = hi.x; v[dr][5] = hi.y; v[dr][6] = hi.z; v[dr][7] = hi.w;
    }
    float m = -INFINITY;
#pragma unroll
    for (int dr = 0; dr < 5; ++dr) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int c = a0 + e;
            if (rok[dr] && c >= j - 2 && c <= j + 2) m = fmaxf(m, v[dr][e]);
        }
    }
    return m;
}

__device__ inline float box_max_any(const float* img, int H, int W, int i, int j, int k) {
    if (k == 2) return (W & 3) == 0 && W >= 8 ? box_max_2v(img, H, W, i, j) : box_max_k<2>(img, H, W, i, j);
    return box_max(img, H, W, i, j, k);
}

// Flux of one band: the box maximum, or with bgw > 0 the box maximum minus
// the mean of the pixels at Chebyshev distance k+1 .. k+bgw inside the image
// (a local background), summed in float64 row by row and rounded once.
__device__ inline float flux_value(const float* img, int H, int W, int i, int j, int k, int bgw) {
    const float m = box_max_any(img, H, W, i, j, k);
    if (bgw <= 0) return m;
    const int r0 = i - k - bgw < 0 ? 0 : i - k - bgw, r1 = i + k + bgw >= H ? H - 1 : i + k + bgw;
    const int c0 = j - k - bgw < 0 ? 0 : j - k - bgw, c1 = j + k + bgw >= W ? W - 1 : j + k + bgw;
    double tot = 0.0;
    int n = 0;
    for (int r = r0; r <= r1; ++r) {
        const int dr = r > i ? r - i : i - r;
        for (int c = c0; c <= c1; ++c) {
            const int dc = c > j ? c - j : j - c;
            if ((dr > dc ? dr : dc) <= k) continue;
            tot += (double)img[(size_t)r * W + c];
            ++n;
        }
    }
    const double mean = n > 0 ? tot / (double)n : 0.0;
    return (float)((double)m - mean);
}

// Current step: every measured source, every band (blocks [0, flux_blocks)),
// and the backward fill of the sources opened at this step (the other
// blocks; their steps precede t by less than the ring length, so the two
// parts write different ring entries).
__device__ void flux_part(const FluxArgs& a, int blk, int nblk);
__device__ void backfill_part(const FluxArgs& a, int blk, int nblk);

__device__ __forceinline__ void flux_block(const FluxArgs& a, int blk, int nblk) {
    if (blk < a.flux_blocks) flux_part(a, blk, a.flux_blocks);
    else backfill_part(a, blk - a.flux_blocks, nblk - a.flux_blocks);
}

__global__ __launch_bounds__(256) void k_flux(FluxArgs a) { flux_block(a, blockIdx.x, gridDim.x); }

// Grouped: context i owns workgroups [start[i], start[i+1]).
__global__ __launch_bounds__(256) void k_flux_group(Grouped<FluxArgs> g) {
    const int i = group_of(g.gi, blockIdx.x);
    flux_block(g.a[i], blockIdx.x - g.gi.start[i], g.gi.start[i + 1] - g.gi.start[i]);
}

// The first entry of each lane is read with the count (used only below it),
// so a lane's box loads follow after one round trip, not three.
__device__ void flux_part(const FluxArgs& a, int blk, int nblk) {
    const int64_t w0 = (int64_t)blk * blockDim.x + threadIdx.x;
    const int n = *a.count;
    const int2 e0 = w0 / a.B < a.cap ? a.list[w0 / a.B] : make_int2(0, 0);
    const int cs = pmod(a.t, a.Tc);
    const uint32_t rej = a.cache_rej[cs];
    const float* frame = a.cache + (size_t)cs * a.plane;
    const int ri = pmod(a.t, kRing);
    const uint32_t allb = (a.B == 32) ? 0xffffffffu : ((1u << a.B) - 1u);
    for (int64_t w = w0; w < (int64_t)n * a.B; w += (int64_t)nblk * blockDim.x) {
        const int2 e = w == w0 ? e0 : a.list[w / a.B];
        const int s = e.x;
        const int b = (int)(w % a.B);
        const float f = ((rej >> b) & 1u)
                            ? 0.0f
                            : flux_value(frame + (size_t)b * a.H * a.W, a.H, a.W, e.y >> 16, e.y & 0xffff,
                                         a.kf, a.bgw);
        a.ring[((size_t)s * a.B + b) * kRing + ri] = f;
        if (b == 0) {
            a.ring_t[(size_t)s * kRing + ri] = a.t;
            a.ring_v[(size_t)s * kRing + ri] = ~rej & allb;
        }
    }
}

// Backward fill of the sources opened at this step.
__device__ void backfill_part(const FluxArgs& a, int blk, int nblk) {
    // steps older than t - (ring length - 1) can lie in no window ending at or
    // after t, and would alias step t in the ring: the fill stops there
    const int T_eff = a.T_bf < kRing - 1 ? a.T_bf : kRing - 1;
    if (T_eff <= 0) return;
    const int64_t per_src = (int64_t)T_eff * a.B;
    const int64_t w0 = (int64_t)blk * blockDim.x + threadIdx.x;
    // the step of an entry follows from its index alone, so the first entry's
    // cache label and QC flags are read with the count and the source, and
    // the box loads come after one round trip
    auto step_of = [&](int64_t w) { return a.t - T_eff + (int)(w % per_src) / a.B; };
    const int n = *a.count_new;
    const int2 e0 = w0 / per_src < a.cap ? a.list_new[w0 / per_src] : make_int2(0, 0);
    const int cs0 = pmod(step_of(w0), a.Tc);
    const int64_t ct0 = a.cache_t[cs0];
    const uint32_t rej0 = a.cache_rej[cs0];
    const uint32_t allb = (a.B == 32) ? 0xffffffffu : ((1u << a.B) - 1u);
    for (int64_t w = w0; w < (int64_t)n * per_src; w += (int64_t)nblk * blockDim.x) {
        const bool first = w == w0;
        const int2 e = first ? e0 : a.list_new[w / per_src];
        const int s = e.x;
        const int b = (int)(w % per_src) % a.B;
        const int64_t tau = step_of(w);
        if (tau < a.t_start) continue;
        const int cs = pmod(tau, a.Tc);
        if ((first ? ct0 : a.cache_t[cs]) != tau) continue;  // step never ingested (gap)
        const uint32_t rej = first ? rej0 : a.cache_rej[cs];
        const float* frame = a.cache + (size_t)cs * a.plane;
        const float f = ((rej >> b) & 1u)
                            ? 0.0f
                            : flux_value(frame + (size_t)b * a.H * a.W, a.H, a.W, e.y >> 16, e.y & 0xffff,
                                         a.kf, a.bgw);
        const int ri = pmod(tau, kRing);
        a.ring[((size_t)s * a.B + b) * kRing + ri] = f;
        if (b == 0) {
            a.ring_t[(size_t)s * kRing + ri] = tau;
            a.ring_v[(size_t)s * kRing + ri] = ~rej & allb;
        }
    }
}

struct WinArgs {
    int n, B;
    const int32_t* slots;     // [n]
    const int64_t* t_end;     // [n] window end per entry (device)
    const float* ring;
    const int64_t* ring_t;
    const uint32_t* ring_v;
    int32_t row_band[kGridRows];  // band on each grid row, -1 if none
    float* out;               // [n][16][64]
};

// Network input windows: x[n][row][c] = F[slot][band(row)][tau], tau = t_end - 63 + c.
__global__ __launch_bounds__(256) void k_windows(WinArgs a) {
    const int64_t total = (int64_t)a.n * kGridRows * kRing;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int n = (int)(w / (kGridRows * kRing));
        const int row = (int)((w / kRing) % kGridRows);
        const int c = (int)(w % kRing);
        const int b = a.row_band[row];
        float v = 0.0f;
        if (b >= 0) {
            const int s = a.slots[n];
            const int64_t tau = a.t_end[n] - (kRing - 1) + c;
            const int ri = pmod(tau, kRing);
            if (a.ring_t[(size_t)s * kRing + ri] == tau && ((a.ring_v[(size_t)s * kRing + ri] >> b) & 1u))
                v = a.ring[((size_t)s * a.B + b) * kRing + ri];
        }
        a.out[w] = v;
    }
}

// Ended list -> (slots, t_end) for the window gather.
__global__ void k_ended_ends(const int32_t* list, const int32_t* count, const int64_t* src_tend,
                             int32_t* slots_out, int64_t* tend_out) {
    const int n = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int s = list[i];
        slots_out[i] = s;
        tend_out[i] = src_tend[s];
    }
}

// Ended episodes of one context appended to a model batch held on the device:
// rows base .. base + take - 1 with base = hdr[0], take = min(n_ended, cap - base).
struct GatherArgs {
    int B, cap, ci;
    const int32_t* list;      // ended slots [n_ended]
    const int32_t* n_ended;
    const int64_t* src_tend;
    const int32_t* src_id;
    const float* ring;
    const int64_t* ring_t;
    const uint32_t* ring_v;
    int32_t row_band[kGridRows];
    int32_t* hdr;
    int first;                // 1: first context of the batch (base 0; block 0 writes the header)
    float* out;               // [cap][16][64]
    int32_t* rows;            // [cap][2]: (context index, id)
};

__global__ __launch_bounds__(256) void k_gather_ended(GatherArgs a) {
    const int base = a.first ? 0 : a.hdr[0];
    const int n_end = *a.n_ended;
    const int room = a.cap - base;
    const int take = n_end < room ? n_end : (room > 0 ? room : 0);
    if (a.first && blockIdx.x == 0 && threadIdx.x < 4)   // no block reads the header in this case
        a.hdr[threadIdx.x] = threadIdx.x == 0 ? take : (threadIdx.x == 1 ? n_end : 0);
    const int64_t total = (int64_t)take * kGridRows * kRing;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(w / (kGridRows * kRing));
        const int row = (int)((w / kRing) % kGridRows);
        const int c = (int)(w % kRing);
        const int s = a.list[e];
        const int b = a.row_band[row];
        float v = 0.0f;
        if (b >= 0) {
            const int64_t tau = a.src_tend[s] - (kRing - 1) + c;
            const int ri = pmod(tau, kRing);
            if (a.ring_t[(size_t)s * kRing + ri] == tau && ((a.ring_v[(size_t)s * kRing + ri] >> b) & 1u))
                v = a.ring[((size_t)s * a.B + b) * kRing + ri];
        }
        a.out[(size_t)(base + e) * kGridRows * kRing + (size_t)row * kRing + c] = v;
        if (row == 0 && c == 0) {
            a.rows[2 * (base + e)] = a.ci;
            a.rows[2 * (base + e) + 1] = a.src_id[s];
        }
    }
}

// hdr[0] += rows taken from this context, hdr[1] += its ended episodes.
__global__ void k_gather_advance(int32_t* hdr, const int32_t* n_ended, int cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int base = hdr[0], n_end = *n_ended;
    const int room = cap - base;
    hdr[0] = base + (n_end < room ? n_end : (room > 0 ? room : 0));
    hdr[1] += n_end;
}

}  // namespace

// Appends context c's ended episodes (as context index ci) to the batch; grid
// sized for up to min(max_sources, cap) windows, counts read on the device.
// The first context of a batch starts the header (one launch); later ones
// read it and advance it in a second launch.
hipError_t launch_gather_ended(lpf_ctx* c, int ci, int32_t* hdr, float* out, int32_t* rows, int cap,
                               hipStream_t s, bool first) {
    GatherArgs a;
    a.B = c->cfg.B;
    a.cap = cap;
    a.ci = ci;
    a.list = c->buf.list_ended;
    a.n_ended = &c->buf.status->n_ended;
    a.src_tend = c->buf.src_tend;
    a.src_id = c->buf.src_id;
    a.ring = c->buf.ring;
    a.ring_t = c->buf.ring_t;
    a.ring_v = c->buf.ring_v;
    for (int r = 0; r < kGridRows; ++r) a.row_band[r] = -1;
    for (int b = 0; b < c->cfg.B; ++b) a.row_band[c->grid_rows[b]] = b;
    a.hdr = hdr;
    a.first = first ? 1 : 0;
    a.out = out;
    a.rows = rows;
    const int most = c->cfg.max_sources < cap ? c->cfg.max_sources : cap;
    int blocks = (int)((((int64_t)most * kGridRows * kRing) + 255) / 256);
    if (blocks > 512) blocks = 512;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_gather_ended, dim3(blocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || first) return e;
    hipLaunchKernelGGL(k_gather_advance, dim3(1), dim3(64), 0, s, hdr, &c->buf.status->n_ended, cap);
    return hipGetLastError();
}

FluxArgs flux_args(lpf_ctx* c, int64_t t) {
    FluxArgs a;
    a.cache = c->buf.cache;
    a.cache_t = c->buf.cache_t;
    a.cache_rej = c->buf.cache_rej;
    a.Tc = c->d.Tc;
    a.B = c->cfg.B;
    a.H = c->cfg.H;
    a.W = c->cfg.W;
    a.kf = c->cfg.flux_halfwidth;
    a.bgw = c->cfg.flux_bg_width;
    a.T_bf = c->cfg.backfill_steps;
    a.t = t;
    a.t_start = c->t_start;
    a.plane = c->d.plane;
    a.ring = c->buf.ring;
    a.ring_t = c->buf.ring_t;
    a.ring_v = c->buf.ring_v;
    a.list = c->buf.list_measured;
    a.count = &c->buf.status->n_measured;
    a.list_new = c->buf.list_new;
    a.count_new = &c->buf.status->n_new;
    a.cap = c->cfg.max_sources;
    a.flux_blocks = 512;
    return a;
}

// Small workgroups: the lanes with work (one per source and band, taken in
// order) then spread over every CU instead of crowding the random box loads
// of a few hundred sources into the miss queues of a hundred CUs.
constexpr int kFluxThreads = 64;
int flux_grid(const FluxArgs& a) { return a.T_bf > 0 ? 1536 : 512; }

hipError_t launch_flux(lpf_ctx* c, int slot, int64_t t) {
    (void)slot;
    const FluxArgs a = flux_args(c, t);
    hipLaunchKernelGGL(k_flux, dim3(flux_grid(a)), dim3(kFluxThreads), 0, c->stream, a);
    return hipGetLastError();
}

hipError_t launch_flux_group(lpf_ctx* const* cs, const int64_t* ts, int n, hipStream_t s) {
    static_assert(sizeof(Grouped<FluxArgs>) <= 4096, "grouped kernel arguments exceed 4 KiB");
    Grouped<FluxArgs> g{};
    g.gi.n = n;
    int total = 0;
    for (int i = 0; i < n; ++i) {
        g.a[i] = flux_args(cs[i], ts[i]);
        g.gi.start[i] = total;
        total += flux_grid(g.a[i]);
    }
    g.gi.start[n] = total;
    hipLaunchKernelGGL(k_flux_group, dim3(total), dim3(kFluxThreads), 0, s, g);
    return hipGetLastError();
}

// Gathers windows for n entries: d_slots[n], d_tend[n] on the device, on stream s.
hipError_t launch_windows_gather(lpf_ctx* c, int n, const int32_t* d_slots, const int64_t* d_tend,
                                 float* d_out, hipStream_t s) {
    WinArgs a;
    a.n = n;
    a.B = c->cfg.B;
    a.slots = d_slots;
    a.t_end = d_tend;
    a.ring = c->buf.ring;
    a.ring_t = c->buf.ring_t;
    a.ring_v = c->buf.ring_v;
    for (int r = 0; r < kGridRows; ++r) a.row_band[r] = -1;
    for (int b = 0; b < c->cfg.B; ++b) a.row_band[c->grid_rows[b]] = b;
    a.out = d_out;
    int blocks = (int)((((int64_t)n * kGridRows * kRing) + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_windows, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ended_ends(lpf_ctx* c, int32_t* slots_out, int64_t* tend_out) {
    hipLaunchKernelGGL(k_ended_ends, dim3(32), dim3(256), 0, c->stream, c->buf.list_ended,
                       &c->buf.status->n_ended, c->buf.src_tend, slots_out, tend_out);
    return hipGetLastError();
}

namespace {

// Boxes of the cached quality-controlled images around (row, col) for the
// steps t_first .. t_first + n - 1: zero outside the image, for a rejected
// band and for a step the cache no longer holds.
__global__ __launch_bounds__(256) void k_cutouts(const float* __restrict__ cache, const int64_t* __restrict__ cache_t,
                                                 const uint32_t* __restrict__ cache_rej, int Tc, int B, int H, int W,
                                                 size_t plane, int row, int col, int half, int64_t t_first, int n,
                                                 float* __restrict__ out) {
    const int side = 2 * half + 1;
    const int64_t total = (int64_t)n * B * side * side;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int dj = (int)(e % side), di = (int)((e / side) % side);
        const int b = (int)((e / ((int64_t)side * side)) % B);
        const int k = (int)(e / ((int64_t)side * side * B));
        const int64_t tau = t_first + k;
        int64_t r = tau % Tc;
        const int slot = (int)(r < 0 ? r + Tc : r);
        const int i = row + di - half, j = col + dj - half;
        float v = 0.0f;
        if (cache_t[slot] == tau && !((cache_rej[slot] >> b) & 1u) && i >= 0 && i < H && j >= 0 && j < W)
            v = cache[(size_t)slot * plane + ((size_t)b * H + i) * W + j];
        out[e] = v;
    }
}

}  // namespace

hipError_t launch_cutouts(lpf_ctx* c, int row, int col, int half, int64_t t_first, int n_steps) {
    const int side = 2 * half + 1;
    const int64_t total = (int64_t)n_steps * c->cfg.B * side * side;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_cutouts, dim3(blocks), dim3(256), 0, c->stream, c->buf.cache, c->buf.cache_t, c->buf.cache_rej,
                       c->d.Tc, c->cfg.B, c->cfg.H, c->cfg.W, c->d.plane, row, col, half, t_first, n_steps,
                       c->buf.cutout);
    return hipGetLastError();
}

}  // namespace lpf
