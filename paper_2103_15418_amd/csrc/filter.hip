// Source detection on one quality-controlled cube (Sec. 2.1.1-2.1.2).
//
// Centre and spread are masked, normalised correlations with the Gaussian
// (or square box) kernel G = g (x) g:
//   C = (G * (W.X)) / (G * W),   S = (G * (W.(X - C)^2)) / (G * W),
// with zero extension outside the image and W = sky mask and not yet
// clipped.  The threshold is y = W-sky and (G*W > 0) and x > c + kappa sqrt(s);
// a peak is a pixel with y = 1 that equals the maximum of x over its
// (2k_p+1)^2 window within the image and the sky mask.
//
// Kernel design (gfx950): one 256-thread workgroup per 64 x 64 output tile
// of one band.  The (64 + 2k)^2 input halo is streamed through LDS in
// 64-row chunks; each chunk is filtered along rows (every thread produces 16
// consecutive outputs from a register window of 16 + 2k values, taps in
// SGPRs), the row results are kept in LDS, and a column pass (16
// consecutive rows per thread) produces the tile.  Inputs come straight from
// HBM (halo re-reads hit L2: tiles are remapped so that each XCD owns a
// contiguous run of tiles).  The epilogue fuses normalisation, threshold and
// the peak test; with one clip iteration neither S nor Y is written to HBM.
//
// Passes for one step (per band not rejected by QC):
//   iteration 1: C  <- filter(M.X) * inv_den          (inv_den static per sky mask)
//                S  <- filter(M.(X-C)^2) * inv_den, threshold, peaks (fused)
//   iteration i > 1 (bands whose mask changed): den <- filter(W), C <- filter(W.X)/den,
//                S <- filter(W.(X-C)^2)/den, Y |= threshold;   then one peak pass.

#include <cmath>
#include <cstdlib>

#include <cstring>

#include "lpf_internal.h"

namespace lpf {
namespace {

constexpr int R = 16;  // outputs per thread per pass

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
template <typename T> struct V8;
template <> struct V8<__bf16> { typedef bf16x8 type; };
template <> struct V8<_Float16> { typedef f16x8 type; };
template <typename T>
__device__ inline floatx4 mfma16(typename V8<T>::type a, typename V8<T>::type b, floatx4 c);
template <>
__device__ inline floatx4 mfma16<__bf16>(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
template <>
__device__ inline floatx4 mfma16<_Float16>(f16x8 a, f16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

enum InMode { IN_MX = 0, IN_ME = 1, IN_W = 2, IN_WX = 3, IN_WE = 4, IN_M = 5, IN_E = 6 };
enum OutMode {
    OUT_C_STATIC = 0,    // C = v * inv_den
    OUT_S_PEAKS = 1,     // S = v * inv_den; threshold; peaks; optional S/Y planes
    OUT_RAW = 2,         // plane = v (den)
    OUT_C_DYN = 3,       // C = v / den
    OUT_S_DYN = 4,       // S = v / den; Y |= threshold; changed flag
    OUT_INV_DEN = 5,     // inv_den = v > 0 ? 1 / v : 0
    OUT_C_E = 6          // C = v * inv_den and E = M (X - C)^2
};

struct FiltArgs {
    const float* X;      // band planes [B][H][W] (cache slot)
    const float* C;      // [B][H][W]
    const uint8_t* M;    // [H][W] or null (all ones)
    const uint8_t* Y;    // [B][H][W] clip mask
    const float* den;    // [B][H][W]
    const float* inv_den;  // [H][W]
    const uint32_t* mbits; // [H][mwords] sky mask, bit j of word w = column 32 w + j (null = all)
    int mwords;
    float* out;          // output plane(s)
    const float* E;      // residual plane M (X - C)^2 (input of IN_E)
    float* E_out;        // residual plane written by OUT_C_E
    int strip_h;         // output rows per strip (strip kernels, multiple of 32)
    float* S_out;        // optional spread plane
    uint8_t* Y_out;      // optional clip plane
    uint8_t* Y_out2;     // optional second clip plane (iteration 1 of several)
    const uint32_t* rej; // rejected bands of this step
    const int32_t* active;  // per-band active flags (null = all)
    int32_t* changed;    // per-band changed flags (OUT_S_DYN / OUT_S_PEAKS with Y plane)
    int32_t* peak_cnt;   // [B]
    int2* cand;          // [B*H*W] above-threshold pixels (pixel index | band << 24, S bits) for the deferred peak test
    int32_t* cand_cnt;   // [1]
    PeakRec* peak_raw;   // [B][cap]
    int peak_cap;
    int kp;              // max-filter half-width
    float kappa;
    int H, W, B;
    int tiles_x, tiles_y;
};

__device__ inline int xcd_remap(int lin, int N) {
    const int nx = 8;
    int q = N / nx, r = N % nx;
    int x = lin % nx, pos = lin / nx;
    return x * q + (x < r ? x : r) + pos;
}

template <int IN>
__device__ inline float load_in(const FiltArgs& a, size_t bo, int gy, int gx) {
    const size_t p = (size_t)gy * a.W + gx;
    float m = a.M ? (float)a.M[p] : 1.0f;
    if (IN == IN_M) return m;
    if (IN == IN_W || IN == IN_WX || IN == IN_WE) {
        if (a.Y[bo + p]) m = 0.0f;
    }
    if (IN == IN_W) return m;
    float x = a.X[bo + p];
    if (IN == IN_MX || IN == IN_WX) return m * x;
    float r = x - a.C[bo + p];
    return m * r * r;
}

// Row window correlation with compile-time half-width K (K > 0) or runtime k (K == 0).
template <int K>
__device__ inline void corr16(const float* src, const Taps& tp, float* acc) {
    if constexpr (K > 0) {
        float w[R + 2 * K];
#pragma unroll
        for (int i = 0; i < R + 2 * K; i += 4) {
            float4 v = *reinterpret_cast<const float4*>(src + i);
            w[i] = v.x;
            if (i + 1 < R + 2 * K) w[i + 1] = v.y;
            if (i + 2 < R + 2 * K) w[i + 2] = v.z;
            if (i + 3 < R + 2 * K) w[i + 3] = v.w;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = 0.0f;
#pragma unroll
        for (int u = 0; u <= 2 * K; ++u) {
            const float g = tp.g[u];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = fmaf(g, w[q + u], acc[q]);
        }
    } else {
        const int k = tp.k;
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = 0.0f;
        for (int u = 0; u <= 2 * k; ++u) {
            const float g = tp.g[u];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = fmaf(g, src[q + u], acc[q]);
        }
    }
}

template <int K>
__device__ inline void corr16_col(const float* src, int stride, const Taps& tp, float* acc) {
    if constexpr (K > 0) {
        float w[R + 2 * K];
#pragma unroll
        for (int i = 0; i < R + 2 * K; ++i) w[i] = src[i * stride];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = 0.0f;
#pragma unroll
        for (int u = 0; u <= 2 * K; ++u) {
            const float g = tp.g[u];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = fmaf(g, w[q + u], acc[q]);
        }
    } else {
        const int k = tp.k;
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = 0.0f;
        for (int u = 0; u <= 2 * k; ++u) {
            const float g = tp.g[u];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = fmaf(g, src[(q + u) * stride], acc[q]);
        }
    }
}

// Local-maximum test (Sec. 2.1.2) with a compile-time half-width: the loads
// of one window row (from clamped, always valid addresses) are issued before
// its comparisons, so a lane pays one memory latency per row rather than per
// pixel, with few registers held (the test runs inside filter epilogues).
template <int KP>
__device__ inline bool is_peak_k(const FiltArgs& a, size_t bo, int y, int x, float xv) {
    constexpr int N = 2 * KP + 1;
    bool peak = true;
#pragma unroll 1
    for (int dy = 0; dy < N; ++dy) {
        const int yy = y + dy - KP;
        if (yy < 0 || yy >= a.H) continue;
        float v[N];
        bool in[N];
#pragma unroll
        for (int dx = 0; dx < N; ++dx) {
            const int xx = x + dx - KP;
            const int xc = xx < 0 ? 0 : (xx >= a.W ? a.W - 1 : xx);
            const size_t p = (size_t)yy * a.W + xc;
            v[dx] = a.X[bo + p];
            in[dx] = xx >= 0 && xx < a.W && (a.M ? a.M[p] != 0 : true);
        }
#pragma unroll
        for (int dx = 0; dx < N; ++dx) peak = peak && !(in[dx] && v[dx] > xv);
    }
    return peak;
}

__device__ inline bool is_peak(const FiltArgs& a, size_t bo, int y, int x, float xv) {
    const int kp = a.kp;
    if (kp == 3) return is_peak_k<3>(a, bo, y, x, xv);   // the paper's 7 x 7 window
    for (int dy = -kp; dy <= kp; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= a.H) continue;
        for (int dx = -kp; dx <= kp; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= a.W) continue;
            const size_t p = (size_t)yy * a.W + xx;
            if (a.M && !a.M[p]) continue;
            if (a.X[bo + p] > xv) return false;
        }
    }
    return true;
}

// Peak test and record append for one above-threshold pixel.
__device__ inline void record_if_peak(const FiltArgs& a, int b, size_t bo, int gy, int gx,
                                                         float xv, float cv, float s) {
    if (!is_peak(a, bo, gy, gx, xv)) return;
    const int idx = atomicAdd(&a.peak_cnt[b], 1);
    if (idx < a.peak_cap) {
        PeakRec rec;
        rec.band = b;
        rec.row = gy;
        rec.col = gx;
        rec.x = xv;
        rec.c = cv;
        rec.s = s;
        rec.sig = (xv - cv) / sqrtf(s);
        a.peak_raw[(size_t)b * a.peak_cap + idx] = rec;
    }
}

// Per-output epilogue: normalisation, threshold, peak test, stores.
template <int OUT>
__device__ inline void epilogue(const FiltArgs& a, int b, size_t bo, int gy, int gx, float v) {
    const size_t p = (size_t)gy * a.W + gx;
    if (OUT == OUT_INV_DEN) {
        a.out[p] = v > 0.0f ? 1.0f / v : 0.0f;
    } else if (OUT == OUT_RAW) {
        a.out[bo + p] = v;
    } else if (OUT == OUT_C_STATIC) {
        a.out[bo + p] = v * a.inv_den[p];
    } else if (OUT == OUT_C_DYN) {
        const float dn = a.den[bo + p];
        a.out[bo + p] = dn > 0.0f ? v / dn : 0.0f;
    } else {
        float s, dpos;
        if (OUT == OUT_S_PEAKS) {
            const float id = a.inv_den[p];
            s = v * id;
            dpos = id;
        } else {
            const float dn = a.den[bo + p];
            s = dn > 0.0f ? v / dn : 0.0f;
            dpos = dn;
        }
        const float cv = a.C[bo + p];
        const float xv = a.X[bo + p];
        const bool m = a.M ? a.M[p] != 0 : true;
        const bool y = m && dpos > 0.0f && xv > cv + a.kappa * sqrtf(s);
        if (a.S_out) a.S_out[bo + p] = s;
        if (OUT == OUT_S_PEAKS) {
            if (a.Y_out) a.Y_out[bo + p] = y ? 1 : 0;
            if (a.Y_out2) a.Y_out2[bo + p] = y ? 1 : 0;
            if (y && is_peak(a, bo, gy, gx, xv)) {
                const int idx = atomicAdd(&a.peak_cnt[b], 1);
                if (idx < a.peak_cap) {
                    PeakRec rec;
                    rec.band = b;
                    rec.row = gy;
                    rec.col = gx;
                    rec.x = xv;
                    rec.c = cv;
                    rec.s = s;
                    rec.sig = (xv - cv) / sqrtf(s);
                    a.peak_raw[(size_t)b * a.peak_cap + idx] = rec;
                }
            }
            if (y && a.changed) a.changed[b] = 1;
        } else {  // OUT_S_DYN: Y_i = Y_{i-1} or y, into the other plane
            const uint8_t old = a.Y[bo + p];
            a.Y_out[bo + p] = (y || old) ? 1 : 0;
            if (y && !old) a.changed[b] = 1;
        }
    }
}

// NQ vertically consecutive outputs (rows gy0 .. gy0+NQ-1, column gx; only the
// first nvalid inside the image).  All loads are issued before any store or
// atomic so their latencies overlap; the common outputs run without branches.
template <int OUT, int NQ>
__device__ inline void epilogue_col(const FiltArgs& a, int b, size_t bo, int gy0, int gx, const float* v,
                                    int nvalid) {
    if (OUT == OUT_C_STATIC) {
        float id[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) id[q] = q < nvalid ? a.inv_den[(size_t)(gy0 + q) * a.W + gx] : 0.0f;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q < nvalid) a.out[bo + (size_t)(gy0 + q) * a.W + gx] = v[q] * id[q];
    } else if (OUT == OUT_C_E) {
        // loads from clamped rows (always inside the image), stores for q < nvalid only
        float id[NQ], xv[NQ], mk[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int gy = gy0 + q < a.H ? gy0 + q : a.H - 1;
            const size_t p = (size_t)gy * a.W + gx;
            id[q] = a.inv_den[p];
            xv[q] = a.X[bo + p];
        }
        if (a.M) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int gy = gy0 + q < a.H ? gy0 + q : a.H - 1;
                mk[q] = (float)a.M[(size_t)gy * a.W + gx];
            }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q) mk[q] = 1.0f;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (q >= nvalid) break;
            const size_t p = bo + (size_t)(gy0 + q) * a.W + gx;
            const float cv = v[q] * id[q];
            const float r = xv[q] - cv;
            a.out[p] = cv;
            a.E_out[p] = mk[q] * r * fabsf(r);   // signed: |E| is the squared residual
        }
    } else if (OUT == OUT_S_PEAKS) {
        float id[NQ], cv[NQ], xv[NQ];
        bool mk[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int gy = gy0 + q < a.H ? gy0 + q : a.H - 1;
            const size_t p = (size_t)gy * a.W + gx;
            id[q] = a.inv_den[p];
            cv[q] = a.C[bo + p];
            xv[q] = a.X[bo + p];
        }
        if (a.M) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int gy = gy0 + q < a.H ? gy0 + q : a.H - 1;
                mk[q] = q < nvalid && a.M[(size_t)gy * a.W + gx] != 0;
            }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q) mk[q] = q < nvalid;
        }
        bool y[NQ];
        float s[NQ];
        bool any = false;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            s[q] = v[q] * id[q];
            y[q] = mk[q] && id[q] > 0.0f && xv[q] > cv[q] + a.kappa * sqrtf(s[q]);
            any |= y[q];
        }
        if (a.S_out || a.Y_out || a.Y_out2) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (q >= nvalid) continue;
                const size_t p = bo + (size_t)(gy0 + q) * a.W + gx;
                if (a.S_out) a.S_out[p] = s[q];
                if (a.Y_out) a.Y_out[p] = y[q] ? 1 : 0;
                if (a.Y_out2) a.Y_out2[p] = y[q] ? 1 : 0;
            }
        }
        if (any) {
            for (int q = 0; q < NQ; ++q)
                if (y[q]) record_if_peak(a, b, bo, gy0 + q, gx, xv[q], cv[q], s[q]);
            if (a.changed) a.changed[b] = 1;
        }
    } else {
        for (int q = 0; q < NQ; ++q)
            if (q < nvalid) epilogue<OUT>(a, b, bo, gy0 + q, gx, v[q]);
    }
}

template <int K, int IN, int OUT>
__global__ __launch_bounds__(kFiltThreads) void k_filter(FiltArgs a, Taps tp) {
    extern __shared__ float lds[];
    const int k = K > 0 ? K : tp.k;
    const int nt = a.tiles_x * a.tiles_y;
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int b = lin / nt;
    const int tile = lin % nt;
    if (OUT != OUT_INV_DEN) {
        if (a.rej && ((*a.rej >> b) & 1u)) return;
        if (a.active && !a.active[b]) return;
    }
    const int ty = tile / a.tiles_x, tx = tile % a.tiles_x;
    const int y0 = ty * kTileH, x0 = tx * kTileW;
    const size_t bo = (size_t)b * a.H * a.W;

    // LDS: stage [64][sw] then rowbuf [(kTileH + 2k)][rw]
    const int sw = ((kTileW + 2 * k + 3) & ~3) + 4;  // float4-aligned rows, skewed
    const int rw = kTileW + 1;
    float* stage = lds;
    float* rowbuf = lds + 64 * sw;
    const int rows_in = kTileH + 2 * k;
    const int tid = threadIdx.x;

    for (int rc = 0; rc < rows_in; rc += 64) {
        const int nr = rows_in - rc < 64 ? rows_in - rc : 64;
        const int wide = kTileW + 2 * k;
        for (int idx = tid; idx < nr * wide; idx += kFiltThreads) {
            const int r = idx / wide, cc = idx - r * wide;
            const int gy = y0 - k + rc + r, gx = x0 - k + cc;
            float v = 0.0f;
            if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) v = load_in<IN>(a, bo, gy, gx);
            stage[r * sw + cc] = v;
        }
        __syncthreads();
        {
            const int r = tid >> 2, cb = (tid & 3) * R;
            if (r < nr) {
                float acc[R];
                corr16<K>(stage + r * sw + cb, tp, acc);
                float* dst = rowbuf + (rc + r) * rw + cb;
#pragma unroll
                for (int q = 0; q < R; ++q) dst[q] = acc[q];
            }
        }
        __syncthreads();
    }

    // Column pass: thread -> column c, rows rb*16 .. rb*16+15.
    const int c = tid & 63, rb = tid >> 6;
    float acc[R];
    corr16_col<K>(rowbuf + (rb * R) * rw + c, rw, tp, acc);
    const int gx = x0 + c;
    if (gx >= a.W) return;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int gy = y0 + rb * R + q;
        if (gy >= a.H) break;
        epilogue<OUT>(a, b, bo, gy, gx, acc[q]);
    }
}

// Fast path (compile-time half-width K, W % 4 == 0): 64-column x 128-row
// tiles, 512 threads.  The row pass reads its 16 + 2K inputs straight from
// global memory as aligned float4 groups into registers (no staging), only
// the row results go through LDS ((128 + 2K) x 65 floats), so three
// workgroups fit on a CU.
constexpr int kTH2 = 128;
constexpr int kThreads2 = 512;

template <int IN>
__device__ inline void load_group(const FiltArgs& a, size_t bo, size_t rowoff, int gx, uint32_t mb4,
                                  float* e) {
    // four consecutive inputs at columns gx..gx+3 (all inside the image);
    // mb4: their sky-mask bits
    const size_t p = rowoff + gx;
    float m0 = (float)(mb4 & 1u), m1 = (float)((mb4 >> 1) & 1u), m2 = (float)((mb4 >> 2) & 1u),
          m3 = (float)((mb4 >> 3) & 1u);
    if (IN == IN_M) {
        e[0] = m0; e[1] = m1; e[2] = m2; e[3] = m3;
        return;
    }
    if (IN == IN_W || IN == IN_WX || IN == IN_WE) {
        const uchar4 yk = *reinterpret_cast<const uchar4*>(a.Y + bo + p);
        if (yk.x) m0 = 0.0f;
        if (yk.y) m1 = 0.0f;
        if (yk.z) m2 = 0.0f;
        if (yk.w) m3 = 0.0f;
    }
    if (IN == IN_W) {
        e[0] = m0; e[1] = m1; e[2] = m2; e[3] = m3;
        return;
    }
    const float4 x = *reinterpret_cast<const float4*>(a.X + bo + p);
    if (IN == IN_MX || IN == IN_WX) {
        e[0] = m0 * x.x; e[1] = m1 * x.y; e[2] = m2 * x.z; e[3] = m3 * x.w;
        return;
    }
    const float4 cc = *reinterpret_cast<const float4*>(a.C + bo + p);
    const float r0 = x.x - cc.x, r1 = x.y - cc.y, r2 = x.z - cc.z, r3 = x.w - cc.w;
    e[0] = m0 * r0 * r0; e[1] = m1 * r1 * r1; e[2] = m2 * r2 * r2; e[3] = m3 * r3 * r3;
}

template <int K, int IN, int OUT>
__global__ __launch_bounds__(kThreads2) void k_filter_fast(FiltArgs a, Taps tp) {
    constexpr int ROWS = kTH2 + 2 * K;        // input rows per tile
    constexpr int RW = kTileW + 1;            // rowbuf stride
    constexpr int SHIFT = (4 - (K % 4)) % 4;  // (x0 - K + cb) mod 4
    constexpr int NV = (SHIFT + R + 2 * K + 3) / 4;  // float4 groups per row task
    __shared__ float rowbuf[ROWS * RW];
    const int nt = a.tiles_x * a.tiles_y;
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int b = lin / nt;
    const int tile = lin % nt;
    if (OUT != OUT_INV_DEN) {
        if (a.rej && ((*a.rej >> b) & 1u)) return;
        if (a.active && !a.active[b]) return;
    }
    const int ty = tile / a.tiles_x, tx = tile % a.tiles_x;
    const int y0 = ty * kTH2, x0 = tx * kTileW;
    const size_t bo = (size_t)b * a.H * a.W;
    const int tid = threadIdx.x;

    // Row pass: task = (input row r, column block cb of 16 outputs).
    for (int task = tid; task < ROWS * 4; task += kThreads2) {
        const int r = task >> 2, cb = (task & 3) * R;
        const int gy = y0 - K + r;
        float acc[R];
        if (gy < 0 || gy >= a.H) {
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = 0.0f;
        } else {
            const size_t rowoff = (size_t)gy * a.W;
            const int a0 = x0 - K + cb - SHIFT;  // multiple of 4
            // sky-mask words covering columns a0 .. a0 + 4 NV - 1
            constexpr int NW = (4 * NV + 31) / 32 + 1;
            const int i0 = a0 >> 5;  // floor division (a0 may be negative)
            uint32_t mw[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int wi = i0 + w;
                mw[w] = !a.mbits ? 0xffffffffu
                                 : (wi >= 0 && wi < a.mwords ? a.mbits[(size_t)gy * a.mwords + wi] : 0u);
            }
            const int sh0 = a0 & 31;
            float v[NV * 4];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int gx = a0 + 4 * j;
                if (gx >= 0 && gx + 3 < a.W) {
                    const int pbit = sh0 + 4 * j;   // bit offset from word i0
                    const int wsel = pbit >> 5;
                    uint32_t wv = mw[0];
#pragma unroll
                    for (int w = 1; w < NW; ++w) wv = wsel == w ? mw[w] : wv;
                    load_group<IN>(a, bo, rowoff, gx, (wv >> (pbit & 31)) & 0xFu, v + 4 * j);
                } else {
                    v[4 * j] = v[4 * j + 1] = v[4 * j + 2] = v[4 * j + 3] = 0.0f;
                }
            }
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = 0.0f;
#pragma unroll
            for (int u = 0; u <= 2 * K; ++u) {
                const float g = tp.g[u];
#pragma unroll
                for (int q = 0; q < R; ++q) acc[q] = fmaf(g, v[SHIFT + q + u], acc[q]);
            }
        }
        float* dst = rowbuf + r * RW + cb;
#pragma unroll
        for (int q = 0; q < R; ++q) dst[q] = acc[q];
    }
    __syncthreads();

    // Column pass: thread -> column c, rows rb*16 .. rb*16+15 (8 row blocks).
    const int c = tid & 63, rb = tid >> 6;
    float w[R + 2 * K];
#pragma unroll
    for (int i = 0; i < R + 2 * K; ++i) w[i] = rowbuf[(rb * R + i) * RW + c];
    float acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0f;
#pragma unroll
    for (int u = 0; u <= 2 * K; ++u) {
        const float g = tp.g[u];
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = fmaf(g, w[q + u], acc[q]);
    }
    const int gx = x0 + c;
    if (gx >= a.W) return;
    // quarters of 4 outputs keep the epilogue's registers below the filter's
    constexpr int EQ = 4;
#pragma unroll
    for (int hf = 0; hf < R / EQ; ++hf) {
        const int gy0 = y0 + rb * R + EQ * hf;
        const int nv = a.H - gy0 < EQ ? (a.H - gy0 > 0 ? a.H - gy0 : 0) : EQ;
        epilogue_col<OUT, EQ>(a, b, bo, gy0, gx, acc + EQ * hf, nv);
    }
}

// 16-bit precision form (bf16 / fp16 operands, float32 accumulation): both
// passes of the separable filter as banded matrix products on
// v_mfma_f32_16x16x32.  For a 16 x 16 output block the row pass is
// In[16 rows][k] x T[k][16], T[k][n] = g[k - n] (0 <= k - n <= 2K), k over the
// 16 + 2K input columns; the column pass is T'[16][k] x RR[k][16] over 16 + 2K
// input rows with the same band.  The taps live in registers for the whole
// tile; the row results are stored transposed (column-major, 16-bit) in LDS
// so each lane's 8 consecutive rows are one 16-byte read.  The epilogue
// (normalisation, threshold, peaks) is the float32 one.
template <typename T, int K, int IN, int OUT>
__global__ __launch_bounds__(kThreads2) void k_filter_mfma(FiltArgs a, Taps tp) {
    typedef typename V8<T>::type vec;
    constexpr int TH = kTH2, TW = kTileW;
    constexpr int NKS = (16 + 2 * K + 31) / 32;                 // 32-wide k steps per block
    constexpr int RNEED = (TH + 2 * K + 15) / 16 * 16;
    constexpr int RCOL = TH - 16 + 32 * NKS;                    // rows the column pass reads
    constexpr int RIN = RNEED > RCOL ? RNEED : RCOL;            // row-pass rows (multiple of 16)
    constexpr int RS = RIN + 8;                                 // LDS stride (elements)
    // fp16 has a narrow range: squared residuals are scaled by 2^-8 and back
    constexpr bool SCALE = sizeof(T) == 2 && !__is_same(T, __bf16) && IN == IN_ME;
    __shared__ T rrt[TW * RS];
    const int nt = a.tiles_x * a.tiles_y;
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int b = lin / nt;
    const int tile = lin % nt;
    if (a.rej && ((*a.rej >> b) & 1u)) return;
    const int ty = tile / a.tiles_x, tx = tile % a.tiles_x;
    const int y0 = ty * TH, x0 = tx * TW;
    const size_t bo = (size_t)b * a.H * a.W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lg = lane >> 4;
    vec tv[NKS];
#pragma unroll
    for (int st = 0; st < NKS; ++st) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = 32 * st + 8 * lg + e - li;
            tv[st][e] = (T)((idx >= 0 && idx <= 2 * K) ? tp.g[idx] : 0.0f);
        }
    }
    // ---- row pass
    for (int blk = wave; blk < (RIN / 16) * (TW / 16); blk += kThreads2 / 64) {
        const int rb = blk / (TW / 16), cb = blk % (TW / 16);
        const int gy = y0 - K + rb * 16 + li;
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        const bool rowin = gy >= 0 && gy < a.H;
        const size_t rowoff = (size_t)(rowin ? gy : 0) * a.W;
#pragma unroll
        for (int st = 0; st < NKS; ++st) {
            const int c0 = x0 + cb * 16 - K + 32 * st + 8 * lg;  // 8 consecutive input columns
            float e8[8];
            uint32_t mb = 0xffu;
            if (a.mbits && rowin) {
                const int w0 = c0 >> 5;
                const uint32_t lo = (w0 >= 0 && w0 < a.mwords) ? a.mbits[(size_t)gy * a.mwords + w0] : 0u;
                const uint32_t hi = (w0 + 1 >= 0 && w0 + 1 < a.mwords) ? a.mbits[(size_t)gy * a.mwords + w0 + 1] : 0u;
                const uint64_t both = ((uint64_t)hi << 32) | lo;
                mb = (uint32_t)(both >> (c0 & 31)) & 0xffu;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int g4 = c0 + 4 * h;
                if (rowin && g4 >= 0 && g4 + 3 < a.W) {
                    if (K % 4 == 0) {
                        load_group<IN>(a, bo, rowoff, g4, (mb >> (4 * h)) & 0xFu, e8 + 4 * h);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const size_t p = rowoff + g4 + q;
                            const float m = (float)((mb >> (4 * h + q)) & 1u);
                            const float x = a.X[bo + p];
                            if (IN == IN_MX) {
                                e8[4 * h + q] = m * x;
                            } else {
                                const float r = x - a.C[bo + p];
                                e8[4 * h + q] = m * r * r;
                            }
                        }
                    }
                } else {
                    e8[4 * h] = e8[4 * h + 1] = e8[4 * h + 2] = e8[4 * h + 3] = 0.0f;
                }
            }
            vec av;
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = (T)(SCALE ? e8[e] * (1.0f / 256.0f) : e8[e]);
            acc = mfma16<T>(av, tv[st], acc);
        }
        // acc[v] = RR[row rb*16 + 4 lg + v][col cb*16 + li] -> transposed LDS
        T* d = rrt + (cb * 16 + li) * RS + rb * 16 + 4 * lg;
#pragma unroll
        for (int v = 0; v < 4; ++v) d[v] = (T)acc[v];
    }
    __syncthreads();
    // ---- column pass + epilogue
    for (int blk = wave; blk < (TH / 16) * (TW / 16); blk += kThreads2 / 64) {
        const int ob = blk / (TW / 16), cb = blk % (TW / 16);
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        const T* src = rrt + (cb * 16 + li) * RS + ob * 16 + 8 * lg;
#pragma unroll
        for (int st = 0; st < NKS; ++st) {
            const vec bv = *reinterpret_cast<const vec*>(src + 32 * st);
            acc = mfma16<T>(tv[st], bv, acc);
        }
        const int gx = x0 + cb * 16 + li;
        if (gx >= a.W) continue;
        const int gy0 = y0 + ob * 16 + 4 * lg;
        float vv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) vv[v] = SCALE ? acc[v] * 256.0f : acc[v];
        epilogue_col<OUT, 4>(a, b, bo, gy0, gx, vv, a.H - gy0 < 4 ? (a.H - gy0 > 0 ? a.H - gy0 : 0) : 4);
    }
}

// Spread epilogue of the strip kernels (four vertically consecutive outputs).
// The residual plane holds E = M r |r| with r = x - C, so the threshold
// x > C + kappa sqrt(S) (kappa >= 0) is E > 0 and E > kappa^2 S, read from
// E at the output pixel: this workgroup loaded it as filter input moments
// ago, so it comes from cache, where X and C would come from HBM.  The 7 x 7
// local-maximum test of the (few) above-threshold pixels is deferred to the
// catalogue kernel through a per-band list that can hold every pixel, so the
// filter kernel neither waits on the window loads nor holds their registers.
__device__ inline void strip_spread_epilogue(const FiltArgs& a, int b, size_t bo, int gy0, int gx, const float* v,
                                             int nvalid) {
    float id[4], ev[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int gy = gy0 + q < a.H ? gy0 + q : a.H - 1;
        const size_t p = (size_t)gy * a.W + gx;
        id[q] = a.inv_den[p];
        ev[q] = a.E[bo + p];   // 0 outside the sky mask
    }
    const float k2 = a.kappa * a.kappa;
    bool y[4];
    float s[4];
    bool any = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        s[q] = v[q] * id[q];
        y[q] = q < nvalid && id[q] > 0.0f && ev[q] > 0.0f && ev[q] > k2 * s[q];
        any |= y[q];
    }
    if (a.S_out || a.Y_out || a.Y_out2) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= nvalid) continue;
            const size_t p = bo + (size_t)(gy0 + q) * a.W + gx;
            if (a.S_out) a.S_out[p] = s[q];
            if (a.Y_out) a.Y_out[p] = y[q] ? 1 : 0;
            if (a.Y_out2) a.Y_out2[p] = y[q] ? 1 : 0;
        }
    }
    if (!any) return;
    if (a.peak_cap > 0) {
        for (int q = 0; q < 4; ++q) {
            if (!y[q]) continue;
            // one list for all bands (< B H W entries: each pixel is listed
            // once); pixel index < 2^24 (H, W <= 4096), band in the top bits
            const int idx = atomicAdd(a.cand_cnt, 1);
            a.cand[idx] = make_int2(((gy0 + q) * a.W + gx) | (b << 24), __float_as_int(s[q]));
        }
    }
    if (a.changed) a.changed[b] = 1;
}

// Strip kernel (float32 path; compile-time half-width K; W % 4 == 0).
// One 256-thread workgroup walks down a 64-column strip of one band in
// chunks of 32 output rows, so every input row is row-filtered once per strip
// (plus 2K warm-up rows) instead of once per tile.  Both passes of the
// separable filter are banded (Toeplitz) products on v_mfma_f32_16x16x4f32,
// float32 operands and accumulation:
//   row pass    Out[16 rows][16 cols] = In[16][k] x T[k][16],   T[k][n] = g[k - n]
//   column pass Out[16 rows][16 cols] = T'[16][k] x R[k][16],   T'[m][k] = g[k - m]
// Lane group q of the instruction owns k = q S .. q S + S - 1, so every lane
// reads its operand as S / 4 aligned 16-byte LDS loads and keeps its S taps in
// registers for the whole strip.  Per 32-row input batch:
//   * coalesced float4 loads, issued one batch ahead into registers, masked
//     and written to an LDS stage;
//   * row pass from the stage into a column-major ring of NB batches of row
//     results (each lane writes its four rows of one column as one 16-byte
//     store; the column pass reads four rows of one column the same way);
//   * column pass for the chunk whose rows are complete; each lane ends with
//     four consecutive rows of one column for the fused epilogue.
// The vector ALUs only stage, normalise, threshold and test peaks.
template <int K>
struct StripGeo {
    static constexpr int SHIFT = (4 - K % 4) % 4;                  // stage col 0 = x0 - K - SHIFT
    static constexpr int S = (16 + 2 * K + SHIFT + 15) / 16 * 4;   // row pass: k per lane group
    static constexpr int SC = (16 + 2 * K + 15) / 16 * 4;          // column pass: k per lane group
    static constexpr int LW = 48 + 4 * S;                          // staged columns
    static constexpr int SW = LW + 4;                              // stage row stride (floats)
    static constexpr int NB = (16 + 4 * SC + 31) / 32;             // ring depth (32-row batches)
    static constexpr int RING = NB * 32;                           // ring rows
    static constexpr int RT = RING + 4;                            // ring column stride (floats)
    static constexpr int NF = 32 * LW / 4;                         // float4 per batch
    static constexpr int NL = (NF + 255) / 256;                    // float4 per thread
    static constexpr int LDS_FLOATS = 32 * SW + kTileW * RT;
};
constexpr int kStripThreads = 256;

// Workgroup lin of one context's launch (band-major over strips and tiles).
template <int K, int IN, int OUT>
__device__ __forceinline__ void strip_body(const FiltArgs& a, const Taps& tp, int lin, float* lds) {
    typedef StripGeo<K> G;
    float* stage = lds;
    float* ring = lds + 32 * G::SW;   // [64 columns][RT]
    // band-minor order: an XCD's contiguous range of lin (xcd_remap) covers one
    // region of the image in every band, so the planes all bands read
    // (1/(G*M), the mask bits) come from that XCD's L2 after the first band
    const int b = lin % a.B;
    const int rem = lin / a.B;
    if (a.rej && ((*a.rej >> b) & 1u)) return;
    const int sy = rem / a.tiles_x, tx = rem % a.tiles_x;
    const int x0 = tx * kTileW;
    const int ys = sy * a.strip_h;
    const int ye = ys + a.strip_h < a.H ? ys + a.strip_h : a.H;
    const size_t bo = (size_t)b * a.H * a.W;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63, li = lane & 15, lq = lane >> 4;
    const float* src = IN == IN_E ? a.E : a.X;

    // ---- batch loads (one batch ahead, in registers)
    float4 pf[G::NL];
    uint32_t pm[G::NL];
    auto prefetch = [&](int bi) {
        const int gy0 = ys - K + 32 * bi;
#pragma unroll
        for (int i = 0; i < G::NL; ++i) {
            const int f = tid + kStripThreads * i;
            pf[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            pm[i] = 0u;
            if (f < G::NF) {
                const int row = f / (G::LW / 4), c4 = f % (G::LW / 4);
                const int gy = gy0 + row, gx = x0 - K - G::SHIFT + 4 * c4;
                if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
                    pf[i] = *reinterpret_cast<const float4*>(src + bo + (size_t)gy * a.W + gx);
                    if (IN == IN_MX) pm[i] = a.mbits ? a.mbits[(size_t)gy * a.mwords + (gx >> 5)] : 0xffffffffu;
                }
            }
        }
    };
    auto stage_write = [&]() {
#pragma unroll
        for (int i = 0; i < G::NL; ++i) {
            const int f = tid + kStripThreads * i;
            if (f < G::NF) {
                const int row = f / (G::LW / 4), c4 = f % (G::LW / 4);
                float4 v = pf[i];
                if (IN == IN_MX) {
                    const int gx = x0 - K - G::SHIFT + 4 * c4;
                    const uint32_t bits = pm[i] >> (gx & 31);
                    v.x = (float)(bits & 1u) * v.x;
                    v.y = (float)((bits >> 1) & 1u) * v.y;
                    v.z = (float)((bits >> 2) & 1u) * v.z;
                    v.w = (float)((bits >> 3) & 1u) * v.w;
                }
                if (IN == IN_E) {   // the residual plane is signed
                    v.x = fabsf(v.x);
                    v.y = fabsf(v.y);
                    v.z = fabsf(v.z);
                    v.w = fabsf(v.w);
                }
                *reinterpret_cast<float4*>(stage + row * G::SW + 4 * c4) = v;
            }
        }
    };

    // taps in registers: B operand of the row pass, A operand of the column pass
    // (with no shift and equal k ranges both passes use the same taps)
    constexpr bool kSameTaps = G::S == G::SC && G::SHIFT == 0;
    float tap[G::S], tapc[G::SC];
#pragma unroll
    for (int s = 0; s < G::S; ++s) {
        const int u = lq * G::S + s - G::SHIFT - li;
        tap[s] = (u >= 0 && u <= 2 * K) ? tp.g[u] : 0.0f;
    }
#pragma unroll
    for (int s = 0; s < G::SC; ++s) {
        const int u = lq * G::SC + s - li;
        tapc[s] = kSameTaps ? 0.0f : ((u >= 0 && u <= 2 * K) ? tp.g[u] : 0.0f);
    }

    // ---- row pass: wave wv owns columns 16 wv .. 16 wv + 15 of both 16-row halves
    auto row_pass = [&](int bi) {
        const int slot = bi % G::NB;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            const float* sp = stage + (rb * 16 + li) * G::SW + wv * 16 + lq * G::S;
#pragma unroll
            for (int p4 = 0; p4 < G::S / 4; ++p4) {
                const float4 av = *reinterpret_cast<const float4*>(sp + 4 * p4);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, tap[4 * p4 + 0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, tap[4 * p4 + 1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, tap[4 * p4 + 2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, tap[4 * p4 + 3], acc, 0, 0, 0);
            }
            // acc[v] = row result of batch row rb*16 + 4 lq + v at column 16 wv + li
            float* dst = ring + (wv * 16 + li) * G::RT + slot * 32 + rb * 16 + 4 * lq;
            *reinterpret_cast<float4*>(dst) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        }
    };

    // ---- column pass for chunk j: wave wv owns columns 16 wv .. +15, both 16-row halves
    auto col_pass = [&](int j) {
        const int gx = x0 + wv * 16 + li;
        floatx4 acc[2];
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) {
            acc[ob] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            const float* cp = ring + (wv * 16 + li) * G::RT;
            const int r0 = 32 * j + ob * 16 + lq * G::SC;     // relative ring row of this lane's k range
#pragma unroll
            for (int p4 = 0; p4 < G::SC / 4; ++p4) {
                const int rr = (r0 + 4 * p4) % G::RING;
                const float4 bv = *reinterpret_cast<const float4*>(cp + rr);
                const float t0 = kSameTaps ? tap[4 * p4 + 0] : tapc[4 * p4 + 0];
                const float t1 = kSameTaps ? tap[4 * p4 + 1] : tapc[4 * p4 + 1];
                const float t2 = kSameTaps ? tap[4 * p4 + 2] : tapc[4 * p4 + 2];
                const float t3 = kSameTaps ? tap[4 * p4 + 3] : tapc[4 * p4 + 3];
                acc[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(t0, bv.x, acc[ob], 0, 0, 0);
                acc[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(t1, bv.y, acc[ob], 0, 0, 0);
                acc[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(t2, bv.z, acc[ob], 0, 0, 0);
                acc[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(t3, bv.w, acc[ob], 0, 0, 0);
            }
        }
        // acc[ob][v] = output row ys + 32 j + 16 ob + 4 lq + v, column gx
        if (gx >= a.W) return;
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) {
            const int gy0 = ys + 32 * j + 16 * ob + 4 * lq;
            const int nv = ye - gy0 < 4 ? (ye - gy0 > 0 ? ye - gy0 : 0) : 4;
            float v4[4] = {acc[ob][0], acc[ob][1], acc[ob][2], acc[ob][3]};
            if (nv <= 0) continue;
            if (OUT == OUT_S_PEAKS) strip_spread_epilogue(a, b, bo, gy0, gx, v4, nv);
            else epilogue_col<OUT, 4>(a, b, bo, gy0, gx, v4, nv);
        }
    };

    const int nch = (ye - ys + 31) / 32;
    const int nbat = nch + G::NB - 1;
    prefetch(0);
    for (int bi = 0; bi < nbat; ++bi) {
        stage_write();
        __syncthreads();                  // stage complete; ring batch bi % NB no longer read
        if (bi + 1 < nbat) prefetch(bi + 1);
        row_pass(bi);
        __syncthreads();                  // ring holds batches bi - NB + 1 .. bi; stage free
        const int j = bi - (G::NB - 1);
        if (j >= 0) col_pass(j);
    }
}

template <int K, int IN, int OUT>
__global__ __launch_bounds__(kStripThreads) void k_filter_strip(FiltArgs a, Taps tp) {
    __shared__ __attribute__((aligned(16))) float lds[StripGeo<K>::LDS_FLOATS];
    strip_body<K, IN, OUT>(a, tp, xcd_remap(blockIdx.x, gridDim.x), lds);
}

// Grouped launch over contexts with the same taps: the XCD-aware order runs
// over the whole grid, then each workgroup finds its context.
template <int K, int IN, int OUT>
__global__ __launch_bounds__(kStripThreads) void k_filter_strip_group(Grouped<FiltArgs> g, Taps tp) {
    __shared__ __attribute__((aligned(16))) float lds[StripGeo<K>::LDS_FLOATS];
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int i = group_of(g.gi, lin);
    strip_body<K, IN, OUT>(g.a[i], tp, lin - g.gi.start[i], lds);
}

// 16-bit precision form of the strip kernels (bf16 / fp16 operands, float32
// accumulation): the same walk, stage and column-major ring, with 16-bit
// elements and v_mfma_f32_16x16x32 (each lane supplies eight consecutive k,
// one 16-byte LDS read).  Row results are rounded to 16 bits in the ring, as
// in the tile kernel of this form; the epilogue is the float32 one.  fp16
// squared residuals are scaled by 2^-8 on the way in and back after the sum.
template <int K>
struct Strip16Geo {
    static constexpr int SHIFT = (4 - K % 4) % 4;
    static constexpr int KS = (16 + 2 * K + SHIFT + 31) / 32;   // row pass: 32-wide k steps
    static constexpr int KC = (16 + 2 * K + 31) / 32;           // column pass: 32-wide k steps
    static constexpr int LW = 48 + 32 * KS;                     // staged columns
    static constexpr int SW = LW + 8;                           // stage row stride (elements)
    static constexpr int NB = (16 + 32 * KC + 31) / 32;         // ring depth (32-row batches)
    static constexpr int RING = NB * 32;
    static constexpr int RT = RING + 8;                         // ring column stride (elements)
    static constexpr int NF = 32 * LW / 4;                      // float4 loads per batch
    static constexpr int NL = (NF + 255) / 256;
};

template <typename T, int K, int IN, int OUT>
__global__ __launch_bounds__(kStripThreads) void k_filter_strip16(FiltArgs a, Taps tp) {
    typedef Strip16Geo<K> G;
    typedef typename V8<T>::type vec;
    constexpr bool SCALE = !__is_same(T, __bf16) && IN == IN_E;
    __shared__ __attribute__((aligned(16))) T stage[32 * G::SW];
    __shared__ __attribute__((aligned(16))) T ring[kTileW * G::RT];
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int b = lin % a.B;   // band-minor, as in strip_body
    const int rem = lin / a.B;
    if (a.rej && ((*a.rej >> b) & 1u)) return;
    const int sy = rem / a.tiles_x, tx = rem % a.tiles_x;
    const int x0 = tx * kTileW;
    const int ys = sy * a.strip_h;
    const int ye = ys + a.strip_h < a.H ? ys + a.strip_h : a.H;
    const size_t bo = (size_t)b * a.H * a.W;
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63, li = lane & 15, lq = lane >> 4;
    const float* src = IN == IN_E ? a.E : a.X;

    float4 pf[G::NL];
    uint32_t pm[G::NL];
    auto prefetch = [&](int bi) {
        const int gy0 = ys - K + 32 * bi;
#pragma unroll
        for (int i = 0; i < G::NL; ++i) {
            const int f = tid + kStripThreads * i;
            pf[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            pm[i] = 0u;
            if (f < G::NF) {
                const int row = f / (G::LW / 4), c4 = f % (G::LW / 4);
                const int gy = gy0 + row, gx = x0 - K - G::SHIFT + 4 * c4;
                if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
                    pf[i] = *reinterpret_cast<const float4*>(src + bo + (size_t)gy * a.W + gx);
                    if (IN == IN_MX) pm[i] = a.mbits ? a.mbits[(size_t)gy * a.mwords + (gx >> 5)] : 0xffffffffu;
                }
            }
        }
    };
    auto stage_write = [&]() {
#pragma unroll
        for (int i = 0; i < G::NL; ++i) {
            const int f = tid + kStripThreads * i;
            if (f < G::NF) {
                const int row = f / (G::LW / 4), c4 = f % (G::LW / 4);
                float4 v = pf[i];
                if (IN == IN_MX) {
                    const int gx = x0 - K - G::SHIFT + 4 * c4;
                    const uint32_t bits = pm[i] >> (gx & 31);
                    v.x = (float)(bits & 1u) * v.x;
                    v.y = (float)((bits >> 1) & 1u) * v.y;
                    v.z = (float)((bits >> 2) & 1u) * v.z;
                    v.w = (float)((bits >> 3) & 1u) * v.w;
                }
                if (IN == IN_E) {   // the residual plane is signed
                    v.x = fabsf(v.x);
                    v.y = fabsf(v.y);
                    v.z = fabsf(v.z);
                    v.w = fabsf(v.w);
                }
                const float sc = SCALE ? 1.0f / 256.0f : 1.0f;
                T* d = stage + row * G::SW + 4 * c4;
                d[0] = (T)(v.x * sc);
                d[1] = (T)(v.y * sc);
                d[2] = (T)(v.z * sc);
                d[3] = (T)(v.w * sc);
            }
        }
    };

    // taps: B operand of the row pass, A operand of the column pass (8 k per lane
    // and step); with no shift and equal k ranges both passes use the same taps
    constexpr bool kSameTaps = G::KS == G::KC && G::SHIFT == 0;
    vec tap[G::KS], tapc[G::KC];
#pragma unroll
    for (int st = 0; st < G::KS; ++st)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int u = 32 * st + 8 * lq + e - G::SHIFT - li;
            tap[st][e] = (T)((u >= 0 && u <= 2 * K) ? tp.g[u] : 0.0f);
        }
#pragma unroll
    for (int st = 0; st < G::KC; ++st)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int u = 32 * st + 8 * lq + e - li;
            tapc[st][e] = kSameTaps ? (T)0.0f : (T)((u >= 0 && u <= 2 * K) ? tp.g[u] : 0.0f);
        }

    auto row_pass = [&](int bi) {
        const int slot = bi % G::NB;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            const T* sp = stage + (rb * 16 + li) * G::SW + wv * 16 + 8 * lq;
#pragma unroll
            for (int st = 0; st < G::KS; ++st) {
                const vec av = *reinterpret_cast<const vec*>(sp + 32 * st);
                acc = mfma16<T>(av, tap[st], acc);
            }
            // acc[v] = row result of batch row rb*16 + 4 lq + v at column 16 wv + li
            T* dst = ring + (wv * 16 + li) * G::RT + slot * 32 + rb * 16 + 4 * lq;
            dst[0] = (T)acc[0];
            dst[1] = (T)acc[1];
            dst[2] = (T)acc[2];
            dst[3] = (T)acc[3];
        }
    };

    auto col_pass = [&](int j) {
        const int gx = x0 + wv * 16 + li;
        floatx4 acc[2];
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) {
            acc[ob] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            const T* cp = ring + (wv * 16 + li) * G::RT;
#pragma unroll
            for (int st = 0; st < G::KC; ++st) {
                const int rr = (32 * j + ob * 16 + 32 * st + 8 * lq) % G::RING;
                const vec bv = *reinterpret_cast<const vec*>(cp + rr);
                acc[ob] = mfma16<T>(kSameTaps ? tap[st] : tapc[st], bv, acc[ob]);
            }
        }
        if (gx >= a.W) return;
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) {
            const int gy0 = ys + 32 * j + 16 * ob + 4 * lq;
            const int nv = ye - gy0 < 4 ? (ye - gy0 > 0 ? ye - gy0 : 0) : 4;
            if (nv <= 0) continue;
            float v4[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) v4[v] = SCALE ? acc[ob][v] * 256.0f : acc[ob][v];
            if (OUT == OUT_S_PEAKS) strip_spread_epilogue(a, b, bo, gy0, gx, v4, nv);
            else epilogue_col<OUT, 4>(a, b, bo, gy0, gx, v4, nv);
        }
    };

    const int nch = (ye - ys + 31) / 32;
    const int nbat = nch + G::NB - 1;
    prefetch(0);
    for (int bi = 0; bi < nbat; ++bi) {
        stage_write();
        __syncthreads();
        if (bi + 1 < nbat) prefetch(bi + 1);
        row_pass(bi);
        __syncthreads();
        const int j = bi - (G::NB - 1);
        if (j >= 0) col_pass(j);
    }
}

// Peaks after several clip iterations: P = Q and Y from the planes.
__global__ __launch_bounds__(256) void k_peaks_planes(FiltArgs a) {
    const int b = blockIdx.y;
    if (a.rej && ((*a.rej >> b) & 1u)) return;
    const size_t HW = (size_t)a.H * a.W;
    const size_t bo = (size_t)b * HW;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < HW;
         p += (size_t)gridDim.x * blockDim.x) {
        if (!a.Y[bo + p]) continue;
        const int gy = (int)(p / a.W), gx = (int)(p % a.W);
        const float xv = a.X[bo + p];
        if (!is_peak(a, bo, gy, gx, xv)) continue;
        const float cv = a.C[bo + p], s = a.den[bo + p];  // den slot carries S here
        const int idx = atomicAdd(&a.peak_cnt[b], 1);
        if (idx < a.peak_cap) {
            PeakRec rec;
            rec.band = b;
            rec.row = gy;
            rec.col = gx;
            rec.x = xv;
            rec.c = cv;
            rec.s = s;
            rec.sig = (xv - cv) / sqrtf(s);
            a.peak_raw[(size_t)b * a.peak_cap + idx] = rec;
        }
    }
}

// Packs the uint8 sky mask into bits: word w of row i holds columns 32w .. 32w+31.
__global__ void k_pack_mask(const uint8_t* __restrict__ m, uint32_t* __restrict__ bits, int H, int W,
                            int mwords) {
    const int64_t n = (int64_t)H * mwords;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int row = (int)(i / mwords), w = (int)(i % mwords);
        uint32_t v = 0u;
        for (int j = 0; j < 32; ++j) {
            const int col = 32 * w + j;
            if (col < W && m[(size_t)row * W + col]) v |= 1u << j;
        }
        bits[i] = v;
    }
}

__global__ void k_detect_init(int32_t* peak_cnt, int32_t* cand_cnt, int32_t* changed, int n_changed, int B) {
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i < B) peak_cnt[i] = 0;
    if (cand_cnt && i < B) cand_cnt[i] = 0;
    if (i < n_changed) changed[i] = 0;
}

// Marks bands active for the next iteration: active = not rejected and changed.
template <int K, int IN, int OUT>
hipError_t run_filter_t(lpf_ctx* c, const FiltArgs& a, int nbands, const Taps& tp) {
    const int k = tp.k;
    const int sw = ((kTileW + 2 * k + 3) & ~3) + 4;
    const size_t lds = sizeof(float) * (64 * sw + (kTileH + 2 * k) * (kTileW + 1));
    const int nblocks = a.tiles_x * a.tiles_y * nbands;
    auto kern = k_filter<K, IN, OUT>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kFiltThreads), lds, c->stream, a, tp);
    return hipGetLastError();
}

template <int K, int IN, int OUT>
hipError_t run_filter(lpf_ctx* c, const FiltArgs& a, int nbands) {
    return run_filter_t<K, IN, OUT>(c, a, nbands, c->taps);
}

template <int K, int IN, int OUT>
hipError_t run_fast(lpf_ctx* c, FiltArgs a, int nbands) {
    a.tiles_y = (a.H + kTH2 - 1) / kTH2;
    const int nblocks = a.tiles_x * a.tiles_y * nbands;
    hipLaunchKernelGGL((k_filter_fast<K, IN, OUT>), dim3(nblocks), dim3(kThreads2), 0, c->stream, a,
                       c->taps);
    return hipGetLastError();
}

// Strip height: a multiple of 32 rows chosen so that a launch has about
// `target` workgroups, unless overridden for tuning by LPF_STRIP_H.  Taller
// strips repeat fewer warm-up rows; shorter ones give more workgroups.
int strip_height(int H, int tiles_x, int nbands, int target) {
    const char* env = std::getenv("LPF_STRIP_H");
    const int forced = env ? std::atoi(env) : 0;
    const int chunks = (H + 31) / 32;
    if (forced > 0) return ((forced + 31) / 32) * 32;
    const int cols = tiles_x * (nbands > 0 ? nbands : 1);
    int sy = (target + cols - 1) / cols;
    if (sy > chunks) sy = chunks;
    if (sy < 1) sy = 1;
    return 32 * ((chunks + sy - 1) / sy);
}

template <int K, int IN, int OUT>
hipError_t run_strip(lpf_ctx* c, FiltArgs a, int nbands) {
    a.tiles_x = (a.W + kTileW - 1) / kTileW;
    // measured on 16 x 1024^2: both passes are fastest at ~4 workgroups per CU
    // (256-row strips)
    a.strip_h = strip_height(a.H, a.tiles_x, nbands, 1024);
    const int nblocks = a.tiles_x * ((a.H + a.strip_h - 1) / a.strip_h) * nbands;
    hipLaunchKernelGGL((k_filter_strip<K, IN, OUT>), dim3(nblocks), dim3(kStripThreads), 0, c->stream, a,
                       c->taps);
    return hipGetLastError();
}

template <typename T, int K, int IN, int OUT>
hipError_t run_strip16(lpf_ctx* c, FiltArgs a, int nbands) {
    a.tiles_x = (a.W + kTileW - 1) / kTileW;
    a.strip_h = strip_height(a.H, a.tiles_x, nbands, 1024);
    const int nblocks = a.tiles_x * ((a.H + a.strip_h - 1) / a.strip_h) * nbands;
    hipLaunchKernelGGL((k_filter_strip16<T, K, IN, OUT>), dim3(nblocks), dim3(kStripThreads), 0, c->stream, a,
                       c->taps);
    return hipGetLastError();
}

template <typename T, int IN, int OUT>
hipError_t dispatch_strip16(lpf_ctx* c, const FiltArgs& a, int nbands) {
    switch (c->d.k) {
        case 15: return run_strip16<T, 15, IN, OUT>(c, a, nbands);
        case 24: return run_strip16<T, 24, IN, OUT>(c, a, nbands);
        case 36: return run_strip16<T, 36, IN, OUT>(c, a, nbands);
        default: return hipErrorInvalidValue;
    }
}

template <int IN, int OUT>
hipError_t dispatch_strip(lpf_ctx* c, const FiltArgs& a, int nbands) {
    if (c->cfg.filter_precision == LPF_PREC_BF16) return dispatch_strip16<__bf16, IN, OUT>(c, a, nbands);
    if (c->cfg.filter_precision == LPF_PREC_FP16) return dispatch_strip16<_Float16, IN, OUT>(c, a, nbands);
    switch (c->d.k) {
        case 15: return run_strip<15, IN, OUT>(c, a, nbands);
        case 24: return run_strip<24, IN, OUT>(c, a, nbands);
        case 36: return run_strip<36, IN, OUT>(c, a, nbands);
        default: return hipErrorInvalidValue;  // derive() enables strips for these only
    }
}

template <typename T, int K, int IN, int OUT>
hipError_t run_mfma(lpf_ctx* c, FiltArgs a, int nbands) {
    a.tiles_y = (a.H + kTH2 - 1) / kTH2;
    const int nblocks = a.tiles_x * a.tiles_y * nbands;
    hipLaunchKernelGGL((k_filter_mfma<T, K, IN, OUT>), dim3(nblocks), dim3(kThreads2), 0, c->stream, a,
                       c->taps);
    return hipGetLastError();
}

template <typename T, int IN, int OUT>
hipError_t dispatch_mfma(lpf_ctx* c, const FiltArgs& a, int nbands) {
    switch (c->d.k) {
        case 15: return run_mfma<T, 15, IN, OUT>(c, a, nbands);
        case 24: return run_mfma<T, 24, IN, OUT>(c, a, nbands);
        case 36: return run_mfma<T, 36, IN, OUT>(c, a, nbands);
        default: return hipErrorInvalidValue;  // configuration validation prevents this
    }
}

template <int IN, int OUT>
hipError_t dispatch_k(lpf_ctx* c, const FiltArgs& a, int nbands) {
    if ((IN == IN_MX || IN == IN_ME) && c->cfg.filter_precision == LPF_PREC_BF16)
        return dispatch_mfma<__bf16, IN, OUT>(c, a, nbands);
    if ((IN == IN_MX || IN == IN_ME) && c->cfg.filter_precision == LPF_PREC_FP16)
        return dispatch_mfma<_Float16, IN, OUT>(c, a, nbands);
    if (a.W % 4 == 0) {
        switch (c->d.k) {
            case 15: return run_fast<15, IN, OUT>(c, a, nbands);
            case 24: return run_fast<24, IN, OUT>(c, a, nbands);
            case 36: return run_fast<36, IN, OUT>(c, a, nbands);
            default: break;
        }
    }
    return run_filter<0, IN, OUT>(c, a, nbands);
}

FiltArgs base_args(lpf_ctx* c, int slot) {
    FiltArgs a{};
    // detection runs on the PSF-correlated image when the pre-filter is on
    a.X = c->d.pre ? c->buf.pre : c->buf.cache + (size_t)slot * c->d.plane;
    a.C = c->buf.centre;
    a.M = c->d.masked ? c->buf.mask : nullptr;
    a.Y = c->buf.clip;
    a.den = c->buf.den;
    a.inv_den = c->buf.inv_den;
    a.E = c->buf.resid;
    a.mbits = c->d.masked ? c->buf.mask_bits : nullptr;
    a.mwords = c->d.mwords;
    a.rej = c->buf.cache_rej + slot;
    a.peak_cnt = c->buf.peak_cnt;
    a.cand = c->buf.cand;
    a.cand_cnt = c->buf.cand_cnt;
    a.peak_raw = c->buf.peak_raw;
    a.peak_cap = c->cfg.peak_cap;
    a.kp = c->cfg.peak_halfwidth;
    a.kappa = c->cfg.kappa;
    a.H = c->cfg.H;
    a.W = c->cfg.W;
    a.B = c->cfg.B;
    a.tiles_x = (a.W + kTileW - 1) / kTileW;
    a.tiles_y = (a.H + kTileH - 1) / kTileH;
    return a;
}

// Grouped strip pass over contexts sharing K and the taps: each context keeps
// the strip height and workgroup order of its own launch, so its results are
// bitwise those of the per-context launch.
template <int K, int IN, int OUT>
hipError_t run_strip_group(lpf_ctx* const* cs, const FiltArgs* as, int n, hipStream_t s) {
    static_assert(sizeof(Grouped<FiltArgs>) + sizeof(Taps) <= 4096, "grouped kernel arguments exceed 4 KiB");
    Grouped<FiltArgs> g{};
    g.gi.n = n;
    int total = 0;
    for (int i = 0; i < n; ++i) {
        FiltArgs a = as[i];
        a.tiles_x = (a.W + kTileW - 1) / kTileW;
        a.strip_h = strip_height(a.H, a.tiles_x, a.B, 1024);
        g.a[i] = a;
        g.gi.start[i] = total;
        total += a.tiles_x * ((a.H + a.strip_h - 1) / a.strip_h) * a.B;
    }
    g.gi.start[n] = total;
    hipLaunchKernelGGL((k_filter_strip_group<K, IN, OUT>), dim3(total), dim3(kStripThreads), 0, s, g, cs[0]->taps);
    return hipGetLastError();
}

template <int IN, int OUT>
hipError_t dispatch_strip_group(lpf_ctx* const* cs, const FiltArgs* as, int n, hipStream_t s) {
    switch (cs[0]->d.k) {
        case 15: return run_strip_group<15, IN, OUT>(cs, as, n, s);
        case 24: return run_strip_group<24, IN, OUT>(cs, as, n, s);
        case 36: return run_strip_group<36, IN, OUT>(cs, as, n, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_pack_mask(lpf_ctx* c) {
    const int64_t n = (int64_t)c->cfg.H * c->d.mwords;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_pack_mask, dim3(blocks), dim3(256), 0, c->stream, c->buf.mask, c->buf.mask_bits,
                       c->cfg.H, c->cfg.W, c->d.mwords);
    return hipGetLastError();
}

hipError_t launch_inv_den(lpf_ctx* c) {
    FiltArgs a = base_args(c, 0);
    a.M = c->d.masked ? c->buf.mask : nullptr;
    a.out = c->buf.inv_den;
    a.rej = nullptr;
    hipError_t e = dispatch_k<IN_M, OUT_INV_DEN>(c, a, 1);
    if (e != hipSuccess || !c->d.pre) return e;
    a.out = c->buf.inv_den_psf;
    return run_filter_t<0, IN_M, OUT_INV_DEN>(c, a, 1, c->taps_psf);
}

// PSF pre-filter: pre = (G_psf * (M X)) / (G_psf * M) of this step's cube.
hipError_t launch_prefilter(lpf_ctx* c, int slot) {
    FiltArgs a = base_args(c, slot);
    a.X = c->buf.cache + (size_t)slot * c->d.plane;
    a.out = c->buf.pre;
    a.inv_den = c->buf.inv_den_psf;
    return run_filter_t<0, IN_MX, OUT_C_STATIC>(c, a, c->cfg.B, c->taps_psf);
}

// Clip planes: clip[j] = buf.clip + j * plane, j = 0, 1.  Iteration 1 writes
// Y_1 into both; iteration i reads clip[(i-1)&1] and writes clip[i&1] whole.
// A band that stops changing therefore holds equal planes, so the final
// plane clip[iters&1] is its last mask whichever iteration it stopped at.
hipError_t launch_filters(lpf_ctx* c, int slot) {
    const int B = c->cfg.B;
    const int iters = c->cfg.clip_iters;
    const size_t plane = c->d.plane;
    uint8_t* clip0 = c->buf.clip;
    uint8_t* clip1 = c->buf.clip ? c->buf.clip + plane : nullptr;
    hipError_t e;
    if (c->d.pre) {
        StageTimer tm(c, 2);
        if ((e = launch_prefilter(c, slot)) != hipSuccess) return e;
    }
    if (c->d.disk) {
        StageTimer tm(c, 3);
        e = launch_disk_filters(c, base_args(c, slot).X, c->buf.cache_rej + slot, c->stream);
        if (e == hipSuccess && c->ev_centre) e = hipEventRecord(c->ev_centre, c->stream);
        return e;
    }
    FiltArgs a = base_args(c, slot);
    a.out = c->buf.centre;
    a.E_out = c->buf.resid;
    {
        StageTimer tm(c, 2);
        e = c->d.strip ? dispatch_strip<IN_MX, OUT_C_E>(c, a, B) : dispatch_k<IN_MX, OUT_C_STATIC>(c, a, B);
        if (e != hipSuccess) return e;
    }
    if (c->ev_centre && (e = hipEventRecord(c->ev_centre, c->stream)) != hipSuccess) return e;
    StageTimer tm3(c, 3);
    a = base_args(c, slot);
    if (iters == 1) {
        a.S_out = c->d.dyn ? c->buf.spread : nullptr;
        a.Y_out = c->d.dyn ? clip1 : nullptr;
        if (!c->d.strip) return dispatch_k<IN_ME, OUT_S_PEAKS>(c, a, B);
        return dispatch_strip<IN_E, OUT_S_PEAKS>(c, a, B);   // peak test of the candidates: k_catalog
    }
    // Several iterations: S and Y planes are materialised and peaks are
    // listed after the last iteration.
    a.S_out = c->buf.spread;
    a.Y_out = clip0;
    a.Y_out2 = clip1;
    a.changed = c->buf.changed + B;   // changed[1]
    a.peak_cap = 0;                   // no peak records from this pass
    a.kp = 0;
    e = c->d.strip ? dispatch_strip<IN_E, OUT_S_PEAKS>(c, a, B) : dispatch_k<IN_ME, OUT_S_PEAKS>(c, a, B);
    if (e != hipSuccess) return e;
    for (int it = 2; it <= iters; ++it) {
        uint8_t* yin = ((it - 1) & 1) ? clip1 : clip0;
        uint8_t* yout = (it & 1) ? clip1 : clip0;
        const int32_t* act = c->buf.changed + (size_t)(it - 1) * B;
        FiltArgs d = base_args(c, slot);
        d.Y = yin;
        d.active = act;
        d.out = c->buf.den;
        if ((e = dispatch_k<IN_W, OUT_RAW>(c, d, B)) != hipSuccess) return e;
        FiltArgs cc = d;
        cc.out = c->buf.centre;
        if ((e = dispatch_k<IN_WX, OUT_C_DYN>(c, cc, B)) != hipSuccess) return e;
        FiltArgs ss = d;
        ss.out = nullptr;
        ss.S_out = c->buf.spread;
        ss.Y_out = yout;
        ss.changed = c->buf.changed + (size_t)it * B;
        if ((e = dispatch_k<IN_WE, OUT_S_DYN>(c, ss, B)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_detect_init, dim3(1), dim3(64), 0, c->stream, c->buf.peak_cnt,
                       (int32_t*)nullptr, (int32_t*)nullptr, 0, B);
    FiltArgs p = base_args(c, slot);
    p.Y = (iters & 1) ? clip1 : clip0;
    p.den = c->buf.spread;  // k_peaks_planes reads S through the den slot
    const int HW = c->cfg.H * c->cfg.W;
    int gx = (HW + 255) / 256;
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(k_peaks_planes, dim3(gx, B), dim3(256), 0, c->stream, p);
    return hipGetLastError();
}

// Contexts whose filter passes can share one launch: float32 strip kernels,
// one clip iteration, the same half-width and taps.
bool filters_groupable(const lpf_ctx* a, const lpf_ctx* b) {
    auto ok = [](const lpf_ctx* c) {
        return c->d.strip && c->cfg.filter_precision == LPF_PREC_FP32 && c->cfg.clip_iters == 1 && !c->ing_stream;
    };
    return ok(a) && ok(b) && a->d.k == b->d.k && std::memcmp(a->taps.g, b->taps.g, sizeof(a->taps.g)) == 0;
}

// The filter passes of launch_filters for n <= kGroupMax groupable contexts
// (their cubes in cache slots slots[i]) as two grouped launches on stream s.
hipError_t launch_filters_group(lpf_ctx* const* cs, const int* slots, int n, hipStream_t s) {
    FiltArgs as[kGroupMax];
    for (int i = 0; i < n; ++i) {
        lpf_ctx* c = cs[i];
        as[i] = base_args(c, slots[i]);
        as[i].out = c->buf.centre;
        as[i].E_out = c->buf.resid;
    }
    hipError_t e = dispatch_strip_group<IN_MX, OUT_C_E>(cs, as, n, s);
    if (e != hipSuccess) return e;
    for (int i = 0; i < n; ++i) {
        lpf_ctx* c = cs[i];
        as[i] = base_args(c, slots[i]);
        as[i].S_out = c->d.dyn ? c->buf.spread : nullptr;
        as[i].Y_out = c->d.dyn ? c->buf.clip + c->d.plane : nullptr;
    }
    return dispatch_strip_group<IN_E, OUT_S_PEAKS>(cs, as, n, s);
}

}  // namespace lpf
