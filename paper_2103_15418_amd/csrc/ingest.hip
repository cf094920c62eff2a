// Quality control of one image cube (App. A) and its entry into the image
// cache (Sec. 2.2, "measure from cached images").
//
// One streaming pass per cube (k_ingest) reads each pixel once and
//   * copies it into the cache slot (device input),
//   * accumulates the band sums sum(x), sum(x^2) in float64 and counts
//     non-finite pixels,
//   * scores it against the running per-pixel mean / std of accepted steps
//     (zeta = |x - mean| / std, max per band),
//   * writes the Welford update of (mean, M2) into the band's *other* state
//     buffer.
// A one-workgroup kernel (k_qc_decide, a wave per band) then reduces the
// per-block partials in a fixed order, forms the robust z-scores of band means and RMS (median /
// median absolute deviation across bands), takes the decision, and commits
// the speculative Welford update of accepted bands by flipping their buffer
// index.  Rejected bands keep their old statistics and are treated as all
// zeros by every later stage (the cached bytes are left untouched).
//
// HBM traffic per subband-pixel: x 4 B, state read 8 B, state write 8 B,
// cache write 4 B = 24 B, the algorithmic minimum of the stage.

#include <cmath>

#include "lpf_internal.h"

namespace lpf {
namespace {

constexpr int kIngThreads = 256;

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wave_max_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

struct PixAcc {
    double sx = 0.0, sxx = 0.0;
    int nf = 0;
    float zmax = 0.0f;
};

__device__ inline void pixel_step(float x, float mu, float m2, bool score, float inv_nm1,
                                  float inv_n1, PixAcc& a, float& mu_out, float& m2_out) {
    double xd = (double)x;
    a.sx += xd;
    a.sxx += xd * xd;
    a.nf += isfinite(x) ? 0 : 1;
    float d = x - mu;
    if (score) {
        float s2 = m2 * inv_nm1;
        if (s2 > 0.0f) a.zmax = fmaxf(a.zmax, fabsf(d) / sqrtf(s2));
    }
    float mu1 = fmaf(d, inv_n1, mu);
    mu_out = mu1;
    m2_out = fmaf(d, x - mu1, m2);
}

// Arguments of one context's ingest pass.
struct IngArgs {
    const float* src;        // the cube [B][H][W] (device), or the cache slot itself
    float* cache_slot;       // [B][H][W]
    const float* wf_mean;    // [2][B][H][W]
    const float* wf_m2;
    float* wf_mean_w;
    float* wf_m2_w;
    const int32_t* wf_n;     // [B]
    const int32_t* wf_cur;   // [B]
    const uint8_t* mask;     // [H][W] or null
    size_t HW, plane;
    int64_t chunk;           // pixels per block
    int warm;
    int nblk;                // blocks per band
    BandPartial* partials;   // [B][nblk]
};

// Block (blk, b) of one context handles pixels [blk*chunk, min(HW, (blk+1)*chunk)) of band b.
template <bool COPY, bool VEC>
__device__ __forceinline__ void ingest_block(const IngArgs& ga, int blk, int b) {
    const float* __restrict__ src = ga.src;
    float* __restrict__ cache_slot = ga.cache_slot;
    const float* __restrict__ wf_mean = ga.wf_mean;
    const float* __restrict__ wf_m2 = ga.wf_m2;
    float* __restrict__ wf_mean_w = ga.wf_mean_w;
    float* __restrict__ wf_m2_w = ga.wf_m2_w;
    const int32_t* __restrict__ wf_n = ga.wf_n;
    const int32_t* __restrict__ wf_cur = ga.wf_cur;
    const uint8_t* __restrict__ mask = ga.mask;
    const size_t HW = ga.HW, plane = ga.plane;
    const int64_t chunk = ga.chunk;
    const int warm = ga.warm;
    BandPartial* __restrict__ partials = ga.partials;
    const int n = wf_n[b];
    const int cur = wf_cur[b];
    const bool armed = n >= warm && n >= 2;
    const float inv_nm1 = armed ? 1.0f / (float)(n - 1) : 0.0f;
    const float inv_n1 = 1.0f / (float)(n + 1);
    const size_t boff = (size_t)b * HW;
    const float* xs = src + boff;
    float* xc = cache_slot + boff;
    const float* mi = wf_mean + (size_t)cur * plane + boff;
    const float* qi = wf_m2 + (size_t)cur * plane + boff;
    float* mo = wf_mean_w + (size_t)(1 - cur) * plane + boff;
    float* qo = wf_m2_w + (size_t)(1 - cur) * plane + boff;
    const size_t p0 = (size_t)blk * chunk;
    const size_t p1 = p0 + chunk < HW ? p0 + chunk : HW;
    PixAcc a;
    if (VEC) {
        // HW % 4 == 0 and chunk % 4 == 0: every float4 is aligned and whole.
        for (size_t p = p0 + 4 * threadIdx.x; p < p1; p += 4 * kIngThreads) {
            float4 x = *reinterpret_cast<const float4*>(xs + p);
            float4 mu = *reinterpret_cast<const float4*>(mi + p);
            float4 m2 = *reinterpret_cast<const float4*>(qi + p);
            uchar4 mk = mask ? *reinterpret_cast<const uchar4*>(mask + p) : make_uchar4(1, 1, 1, 1);
            if (COPY) *reinterpret_cast<float4*>(xc + p) = x;
            float4 mu1, q1;
            pixel_step(x.x, mu.x, m2.x, armed && mk.x, inv_nm1, inv_n1, a, mu1.x, q1.x);
            pixel_step(x.y, mu.y, m2.y, armed && mk.y, inv_nm1, inv_n1, a, mu1.y, q1.y);
            pixel_step(x.z, mu.z, m2.z, armed && mk.z, inv_nm1, inv_n1, a, mu1.z, q1.z);
            pixel_step(x.w, mu.w, m2.w, armed && mk.w, inv_nm1, inv_n1, a, mu1.w, q1.w);
            *reinterpret_cast<float4*>(mo + p) = mu1;
            *reinterpret_cast<float4*>(qo + p) = q1;
        }
    } else {
        for (size_t p = p0 + threadIdx.x; p < p1; p += kIngThreads) {
            float x = xs[p];
            if (COPY) xc[p] = x;
            bool mk = mask ? mask[p] != 0 : true;
            float mu1, q1;
            pixel_step(x, mi[p], qi[p], armed && mk, inv_nm1, inv_n1, a, mu1, q1);
            mo[p] = mu1;
            qo[p] = q1;
        }
    }
    // Fixed-shape block reduction (deterministic).
    __shared__ double s_sx[kIngThreads / 64], s_sxx[kIngThreads / 64];
    __shared__ int s_nf[kIngThreads / 64];
    __shared__ float s_z[kIngThreads / 64];
    double sx = wave_sum_d(a.sx), sxx = wave_sum_d(a.sxx);
    int nf = wave_sum_i(a.nf);
    float z = wave_max_f(a.zmax);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s_sx[w] = sx;
        s_sxx[w] = sxx;
        s_nf[w] = nf;
        s_z[w] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        BandPartial bp;
        bp.sx = 0.0;
        bp.sxx = 0.0;
        bp.nonfinite = 0;
        bp.zmax = 0.0f;
        for (int i = 0; i < kIngThreads / 64; ++i) {
            bp.sx += s_sx[i];
            bp.sxx += s_sxx[i];
            bp.nonfinite += s_nf[i];
            bp.zmax = fmaxf(bp.zmax, s_z[i]);
        }
        bp.pad[0] = bp.pad[1] = 0;
        partials[(size_t)b * ga.nblk + blk] = bp;
    }
}

// grid: (nblk, B), one context.
template <bool COPY, bool VEC>
__global__ __launch_bounds__(kIngThreads) void k_ingest(IngArgs a) {
    ingest_block<COPY, VEC>(a, blockIdx.x, blockIdx.y);
}

// Grouped launch over several contexts: context i owns the flat blocks
// [start[i], start[i+1]) = nblk_i x B_i of them, band-major.
template <bool COPY, bool VEC>
__global__ __launch_bounds__(kIngThreads) void k_ingest_group(Grouped<IngArgs> g) {
    const int i = group_of(g.gi, blockIdx.x);
    const IngArgs& a = g.a[i];
    const int local = blockIdx.x - g.gi.start[i];
    ingest_block<COPY, VEC>(a, local % a.nblk, local / a.nblk);
}

__device__ inline double readlane_d(double v, int j) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), j);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), j);
    return __hiloint2double(hi, lo);
}

// Median of the entries of v flagged in use, over lanes 0..B-1 of one fully
// active wave: each lane ranks its value (ties by index) against the others
// read lane by lane from registers, and the median is read from the lanes
// that hold the middle ranks.  Every lane returns it.
__device__ double wave_median(double v, bool use, int B) {
    const int lane = threadIdx.x & 63;
    const bool u = use && lane < B;
    const uint64_t um = __ballot(u);
    const int m = __popcll(um);
    if (m == 0) return 0.0;
    int rank = 0;
    for (int j = 0; j < B; ++j) {
        if (!((um >> j) & 1ull)) continue;   // uniform
        const double vj = readlane_d(v, j);
        rank += (vj < v || (vj == v && j < lane)) ? 1 : 0;
    }
    const uint64_t hi = __ballot(u && rank == m / 2);
    const double vh = readlane_d(v, __ffsll((unsigned long long)hi) - 1);
    if (m & 1) return vh;
    const uint64_t lo = __ballot(u && rank == m / 2 - 1);
    return 0.5 * (readlane_d(v, __ffsll((unsigned long long)lo) - 1) + vh);
}

// Robust z of lane b's value: (v - med) / max(MAD, floor |med|), 0 if unused.
__device__ double wave_robust_z(double v, bool use, int B, double floor_rel) {
    const double med = wave_median(v, use, B);
    double mad = wave_median(fabs(v - med), use, B);
    const double fl = floor_rel * fabs(med);
    if (fl > mad) mad = fl;
    if (!use) return 0.0;
    const double dlt = v - med;
    return mad > 0.0 ? dlt / mad : (dlt == 0.0 ? 0.0 : INFINITY);
}

struct QcParams {
    int B;
    int nblk;
    double npix;
    double band_z, rms_z, rms_floor, zeta;
    int warm;
    const BandPartial* partials;
    int32_t* wf_n;
    int32_t* wf_cur;
    double* bandstats;
    int64_t* cache_t;
    uint32_t* cache_rej;
    int slot;
    int64_t t;
    DevStatus* status;
};

// One wave per band reduces that band's block partials (lane l sums blocks
// l, l+64, ... in order, then a fixed butterfly), then lane 0 of the block
// takes the decision.  One workgroup of 64 B_max threads per context.
__device__ __forceinline__ void qc_decide(const QcParams& q) {
    __shared__ double s_mean[kMaxB], s_rms[kMaxB];
    __shared__ int s_nf[kMaxB];
    __shared__ float s_z[kMaxB];
    const int b = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (b < q.B) {
        double sx = 0.0, sxx = 0.0;
        int nf = 0;
        float z = 0.0f;
        const BandPartial* p = q.partials + (size_t)b * q.nblk;
        for (int i = lane; i < q.nblk; i += 64) {
            sx += p[i].sx;
            sxx += p[i].sxx;
            nf += p[i].nonfinite;
            z = fmaxf(z, p[i].zmax);
        }
        sx = wave_sum_d(sx);
        sxx = wave_sum_d(sxx);
        nf = wave_sum_i(nf);
        z = wave_max_f(z);
        if (lane == 0) {
            s_mean[b] = sx / q.npix;
            s_rms[b] = sqrt(sxx / q.npix);
            s_nf[b] = nf;
            s_z[b] = z;
        }
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;   // the decision: lanes 0..B-1 of wave 0
    const int i = threadIdx.x;
    const bool in = i < q.B;
    const bool ok = in && s_nf[i] == 0;
    const double zm = wave_robust_z(in ? s_mean[i] : 0.0, ok, q.B, 0.0);
    const double zr = q.rms_z > 0.0 ? wave_robust_z(in ? s_rms[i] : 0.0, ok, q.B, q.rms_floor) : 0.0;
    bool bad = false;
    if (in) {
        const int n = q.wf_n[i];
        const bool armed = n >= q.warm && n >= 2;
        bad = !ok || fabs(zm) > q.band_z || (q.rms_z > 0.0 && fabs(zr) > q.rms_z) ||
              (armed && (double)s_z[i] > q.zeta);
        double* bs = q.bandstats + 6 * i;
        bs[0] = s_mean[i];
        bs[1] = s_rms[i];
        bs[2] = zm;
        bs[3] = zr;
        bs[4] = armed ? (double)s_z[i] : 0.0;
        bs[5] = (double)s_nf[i];
        if (!bad) {  // commit the speculative Welford update
            q.wf_n[i] = n + 1;
            q.wf_cur[i] = 1 - q.wf_cur[i];
        }
    }
    const uint64_t bal = __ballot(bad);
    const uint32_t rej = (uint32_t)(bal & 0xffffffffull);
    if (i != 0) return;
    q.cache_t[q.slot] = q.t;
    q.cache_rej[q.slot] = rej;
    q.status->rejected = rej;
}

__global__ __launch_bounds__(1024) void k_qc_decide(QcParams q) { qc_decide(q); }

// Grouped: workgroup i decides for context i.
__global__ __launch_bounds__(1024) void k_qc_decide_group(Grouped<QcParams> g) { qc_decide(g.a[blockIdx.x]); }

}  // namespace

IngArgs ingest_args(lpf_ctx* c, const float* src, int slot) {
    const auto& d = c->d;
    IngArgs a;
    a.src = src;
    a.cache_slot = c->buf.cache + (size_t)slot * d.plane;
    a.wf_mean = c->buf.wf_mean;
    a.wf_m2 = c->buf.wf_m2;
    a.wf_mean_w = c->buf.wf_mean;
    a.wf_m2_w = c->buf.wf_m2;
    a.wf_n = c->buf.wf_n;
    a.wf_cur = c->buf.wf_cur;
    a.mask = d.masked ? c->buf.mask : nullptr;
    a.HW = d.HW;
    a.plane = d.plane;
    a.chunk = (int64_t)((d.HW + d.nblk - 1) / d.nblk + 3) / 4 * 4;
    a.warm = c->cfg.qc_warmup;
    a.nblk = d.nblk;
    a.partials = c->buf.partials;
    return a;
}

hipError_t launch_ingest(lpf_ctx* c, const float* src, bool copy, int slot, hipStream_t s) {
    const IngArgs a = ingest_args(c, src, slot);
    const bool vec = (c->d.HW % 4) == 0;
    dim3 grid(c->d.nblk, c->cfg.B);
    if (copy && vec) hipLaunchKernelGGL((k_ingest<true, true>), grid, dim3(kIngThreads), 0, s, a);
    else if (copy) hipLaunchKernelGGL((k_ingest<true, false>), grid, dim3(kIngThreads), 0, s, a);
    else if (vec) hipLaunchKernelGGL((k_ingest<false, true>), grid, dim3(kIngThreads), 0, s, a);
    else hipLaunchKernelGGL((k_ingest<false, false>), grid, dim3(kIngThreads), 0, s, a);
    return hipGetLastError();
}

// One grouped launch for n <= kGroupMax contexts whose cubes are all on the
// device (copy) or all already in their cache slots, and whose planes are all
// float4-aligned or not (vec); srcs[i] and slots[i] as in launch_ingest.
hipError_t launch_ingest_group(lpf_ctx* const* cs, const float* const* srcs, const int* slots, int n, bool copy,
                               bool vec, hipStream_t s) {
    static_assert(sizeof(Grouped<IngArgs>) <= 4096, "grouped kernel arguments exceed 4 KiB");
    Grouped<IngArgs> g{};
    g.gi.n = n;
    int total = 0;
    for (int i = 0; i < n; ++i) {
        g.a[i] = ingest_args(cs[i], srcs[i], slots[i]);
        g.gi.start[i] = total;
        total += cs[i]->d.nblk * cs[i]->cfg.B;
    }
    g.gi.start[n] = total;
    if (copy && vec) hipLaunchKernelGGL((k_ingest_group<true, true>), dim3(total), dim3(kIngThreads), 0, s, g);
    else if (copy) hipLaunchKernelGGL((k_ingest_group<true, false>), dim3(total), dim3(kIngThreads), 0, s, g);
    else if (vec) hipLaunchKernelGGL((k_ingest_group<false, true>), dim3(total), dim3(kIngThreads), 0, s, g);
    else hipLaunchKernelGGL((k_ingest_group<false, false>), dim3(total), dim3(kIngThreads), 0, s, g);
    return hipGetLastError();
}

QcParams qc_params(lpf_ctx* c, int slot, int64_t t) {
    QcParams q;
    q.B = c->cfg.B;
    q.nblk = c->d.nblk;
    q.npix = (double)c->d.HW;
    q.band_z = c->cfg.qc_band_z;
    q.rms_z = c->cfg.qc_rms_z;
    q.rms_floor = c->cfg.qc_rms_floor;
    q.zeta = c->cfg.qc_pixel_zeta;
    q.warm = c->cfg.qc_warmup;
    q.partials = c->buf.partials;
    q.wf_n = c->buf.wf_n;
    q.wf_cur = c->buf.wf_cur;
    q.bandstats = c->buf.bandstats;
    q.cache_t = c->buf.cache_t;
    q.cache_rej = c->buf.cache_rej;
    q.slot = slot;
    q.t = t;
    q.status = c->buf.status;
    return q;
}

hipError_t launch_qc_decide(lpf_ctx* c, int slot, int64_t t, hipStream_t s) {
    hipLaunchKernelGGL(k_qc_decide, dim3(1), dim3(64 * c->cfg.B), 0, s, qc_params(c, slot, t));
    return hipGetLastError();
}

hipError_t launch_qc_decide_group(lpf_ctx* const* cs, const int* slots, const int64_t* ts, int n, hipStream_t s) {
    static_assert(sizeof(Grouped<QcParams>) <= 4096, "grouped kernel arguments exceed 4 KiB");
    Grouped<QcParams> g{};
    g.gi.n = n;
    int bmax = 1;
    for (int i = 0; i < n; ++i) {
        g.a[i] = qc_params(cs[i], slots[i], ts[i]);
        g.gi.start[i] = i;
        if (cs[i]->cfg.B > bmax) bmax = cs[i]->cfg.B;
    }
    g.gi.start[n] = n;
    hipLaunchKernelGGL(k_qc_decide_group, dim3(n), dim3(64 * bmax), 0, s, g);
    return hipGetLastError();
}

}  // namespace lpf
