// Circular uniform background kernel (Sec. 2.1.1 names the circular uniform
// kernel as the alternative to the Gaussian): the centre C and spread S are
// means over the offsets with u^2 + v^2 <= k^2 that lie in the image and the
// sky mask, C = (D * (M X)) / (D * M), S = (D * (M (X - C)^2)) / (D * M).
//
// The disk is not separable, but each of its rows is a run of 2 h(u) + 1
// columns with h(u) = floor(sqrt(k^2 - u^2)).  A 256-thread workgroup owns a
// 64 x 32 output tile: it stages the float64 running sums of its 32 + 2k
// input rows (each row's prefix over the 64 + 2k columns the tile needs) in
// LDS, and every output adds the 2k + 1 run sums of its disk, each the
// difference of two prefix values.  Float64 keeps the differences exact to
// far below the float32 result's rounding.  The spread pass ends with the
// threshold x > c + kappa sqrt(s) and lists the pixels above it for the
// catalogue's local-maximum test, as the strip filters do.

#include "lpf_internal.h"

namespace lpf {
namespace {

constexpr int kDiskTW = 64, kDiskTH = 32, kDiskThreads = 256;
constexpr int kDiskMaxK = 32;

struct DiskArgs {
    const float* X;          // [B][H][W] detection image of this step
    const float* C;          // [B][H][W] centre (spread pass)
    const uint8_t* M;        // [H][W] sky mask or null
    const float* inv_den;    // [H][W] 1 / (D * M), 0 where that is 0
    float* out;              // inv_den (den pass) or C (centre pass)
    float* S_out;            // optional spread plane
    uint8_t* Y_out;          // optional threshold plane
    const uint32_t* rej;     // rejected bands of this step
    int2* cand;              // above-threshold pixels (pixel index | band << 24, S bits)
    int32_t* cand_cnt;
    float kappa;
    int H, W, k;
    int tiles_x, tiles_y;
    int h[kDiskMaxK + 1];    // run half-widths h(|u|)
};

enum DiskMode { DISK_DEN = 0, DISK_C = 1, DISK_S = 2 };

template <int MODE>
__global__ __launch_bounds__(kDiskThreads) void k_disk(DiskArgs a) {
    extern __shared__ double P[];   // [32 + 2k][64 + 2k + 1] row prefix sums
    const int k = a.k;
    const int LW = kDiskTW + 2 * k;
    const int PW = LW + 1;
    const int NR = kDiskTH + 2 * k;
    const int nt = a.tiles_x * a.tiles_y;
    const int b = MODE == DISK_DEN ? 0 : (int)blockIdx.x / nt;
    const int tile = (int)blockIdx.x % nt;
    if (MODE != DISK_DEN && a.rej && ((*a.rej >> b) & 1u)) return;
    const int y0 = (tile / a.tiles_x) * kDiskTH, x0 = (tile % a.tiles_x) * kDiskTW;
    const size_t bo = (size_t)b * a.H * a.W;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    // input rows y0 - k .. y0 + 32 + k - 1, columns x0 - k .. x0 + 64 + k - 1 (zero outside)
    for (int r = wv; r < NR; r += kDiskThreads / 64) {
        const int gy = y0 - k + r;
        double carry = 0.0;
        for (int c0 = 0; c0 < LW; c0 += 64) {
            const int j = c0 + lane;
            const int gx = x0 - k + j;
            float v = 0.0f;
            if (j < LW && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
                const size_t p = (size_t)gy * a.W + gx;
                const float m = a.M ? (float)a.M[p] : 1.0f;
                if (MODE == DISK_DEN) {
                    v = m;
                } else if (MODE == DISK_C) {
                    v = m != 0.0f ? a.X[bo + p] : 0.0f;
                } else {
                    const float d = a.X[bo + p] - a.C[bo + p];
                    v = m != 0.0f ? d * d : 0.0f;
                }
            }
            double s = (double)v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const double t = __shfl_up(s, o, 64);
                if (lane >= o) s += t;
            }
            if (j < LW) P[r * PW + j + 1] = carry + s;
            carry += __shfl(s, 63, 64);
        }
        if (lane == 0) P[r * PW] = 0.0;
    }
    __syncthreads();

    const int cx = threadIdx.x & 63;
    const int gx = x0 + cx;
    if (gx >= a.W) return;
    for (int q = 0; q < kDiskTH / 4; ++q) {
        const int row = (threadIdx.x >> 6) + 4 * q;
        const int gy = y0 + row;
        if (gy >= a.H) break;
        double acc = 0.0;
        for (int u = -k; u <= k; ++u) {
            const int hu = a.h[u < 0 ? -u : u];
            const double* pr = P + (row + k + u) * PW;
            acc += pr[cx + k + hu + 1] - pr[cx + k - hu];
        }
        const size_t p = (size_t)gy * a.W + gx;
        if (MODE == DISK_DEN) {
            a.out[p] = acc > 0.0 ? (float)(1.0 / acc) : 0.0f;
        } else if (MODE == DISK_C) {
            a.out[bo + p] = (float)acc * a.inv_den[p];
        } else {
            const float id = a.inv_den[p];
            const float s = (float)acc * id;
            const float x = a.X[bo + p], c = a.C[bo + p];
            const bool in = a.M ? a.M[p] != 0 : true;
            const bool y = in && id > 0.0f && x > c + a.kappa * sqrtf(s);
            if (a.S_out) a.S_out[bo + p] = s;
            if (a.Y_out) a.Y_out[bo + p] = y ? 1 : 0;
            if (y) {
                const int idx = atomicAdd(a.cand_cnt, 1);
                a.cand[idx] = make_int2((int)p | (b << 24), __float_as_int(s));
            }
        }
    }
}

DiskArgs disk_args(lpf_ctx* c) {
    DiskArgs a{};
    a.M = c->d.masked ? c->buf.mask : nullptr;
    a.inv_den = c->buf.inv_den;
    a.kappa = c->cfg.kappa;
    a.H = c->cfg.H;
    a.W = c->cfg.W;
    a.k = c->d.k;
    a.tiles_x = (a.W + kDiskTW - 1) / kDiskTW;
    a.tiles_y = (a.H + kDiskTH - 1) / kDiskTH;
    for (int u = 0; u <= a.k; ++u) {
        int h = 0;
        while ((h + 1) * (h + 1) + u * u <= a.k * a.k) ++h;
        a.h[u] = h;
    }
    return a;
}

template <int MODE>
hipError_t run_disk(const DiskArgs& a, int nbands, hipStream_t s) {
    const size_t lds = sizeof(double) * (size_t)(kDiskTH + 2 * a.k) * (kDiskTW + 2 * a.k + 1);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_disk<MODE>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_disk<MODE>), dim3(a.tiles_x * a.tiles_y * nbands), dim3(kDiskThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace

int disk_max_halfwidth() { return kDiskMaxK; }

// 1 / (D * M) of the geometry (at create).
hipError_t launch_disk_inv_den(lpf_ctx* c) {
    DiskArgs a = disk_args(c);
    a.out = c->buf.inv_den;
    return run_disk<DISK_DEN>(a, 1, c->stream);
}

// Centre pass then spread + threshold pass on the detection image X of this step.
hipError_t launch_disk_filters(lpf_ctx* c, const float* X, const uint32_t* rej, hipStream_t s) {
    DiskArgs a = disk_args(c);
    a.X = X;
    a.rej = rej;
    a.out = c->buf.centre;
    hipError_t e = run_disk<DISK_C>(a, c->cfg.B, s);
    if (e != hipSuccess) return e;
    a.C = c->buf.centre;
    a.out = nullptr;
    a.S_out = c->d.dyn ? c->buf.spread : nullptr;
    a.Y_out = c->d.dyn ? c->buf.clip + c->d.plane : nullptr;
    a.cand = c->buf.cand;
    a.cand_cnt = c->buf.cand_cnt;
    return run_disk<DISK_S>(a, c->cfg.B, s);
}

}  // namespace lpf
