// Parameter-inference network (Sec. 2.3.2-2.3.3) on gfx950 matrix cores.
//
// g(x, W) maps a 1 x 16 x 64 dynamic spectrum to [mu ; L]: four 3x3
// convolutions (1->32->32->64->64, zero padding 1, leaky rectifier
// phi(h) = h >= 0 ? h : alpha h), a dense layer 65536->128 with phi and a
// linear layer 128->14.  mu = out[0:4]; out[4:14] fill the lower-triangular
// Cholesky factor L row by row, its diagonal through softplus so that
// Sigma = L L^T is a valid covariance.
//
// Layout: activations NHWC ([n][row][col][channel]), float32.
// conv1 (one input channel, 9 MACs per output) runs on the vector ALUs.
// conv2..4 are implicit GEMMs (pixels x (3*3*Cin) times (3*3*Cin) x Cout)
// on v_mfma_f32_32x32x2f32: a 256-thread workgroup owns 64 x 64 outputs
// (one image row for Cout = 64, two rows for Cout = 32), stages the three
// (or four) input rows channel-major in LDS and streams weights from L2.
// fc1 is a split-K GEMM on the same instruction (K chunks of 512 staged in
// LDS) with a fixed-order reduction; fc2 and the head run on the ALUs.

#include <cmath>
#include <mutex>

#include "lpf_internal.h"

namespace lpf {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kGH = 16, kGW = 64;
constexpr int kFlat = 64 * kGH * kGW;  // 65536
constexpr int kHidden = 128;
constexpr int kOut = 14;
constexpr int kSplitK = 512;
constexpr int kNSplit = kFlat / kSplitK;  // 128

size_t align64(size_t x) { return (x + 63) & ~size_t(63); }

// element offsets of the 16-bit weight copies
constexpr size_t kW16o2 = 0, kW16o3 = kW16o2 + 9 * 32 * 32, kW16o4 = kW16o3 + 9 * 32 * 64,
                 kW16of1 = kW16o4 + 9 * 64 * 64, kW16total = kW16of1 + (size_t)kFlat * kHidden;



ModelLayout make_layout() {
    ModelLayout L{};
    size_t o = 0;
    L.w1 = o; o = align64(o + 9 * 32);
    L.b1 = o; o = align64(o + 32);
    L.w2 = o; o = align64(o + 9 * 32 * 32);
    L.b2 = o; o = align64(o + 32);
    L.w3 = o; o = align64(o + 9 * 32 * 64);
    L.b3 = o; o = align64(o + 64);
    L.w4 = o; o = align64(o + 9 * 64 * 64);
    L.b4 = o; o = align64(o + 64);
    L.f1 = o; o = align64(o + (size_t)kFlat * kHidden);
    L.fb1 = o; o = align64(o + kHidden);
    L.f2 = o; o = align64(o + kHidden * kOut);
    L.fb2 = o; o = align64(o + kOut);
    L.total = o;
    return L;
}

__device__ inline float act_fn(float v, float alpha) { return v >= 0.0f ? v : alpha * v; }

// Device layout of the float32 fc1 weights W1[k][j] (k < 65536, j < 128):
// groups of eight k, and inside a group (k & 1, (k & 7) >> 1), so that lane
// (m, kk) of a 32x32x2 product reads the B operands of four consecutive
// products, W1[8 g + 2 q + kk][j] for q = 0..3, as one 16-byte load, and the
// 64 lanes of a wave read 1 KB contiguous.
__host__ __device__ inline size_t f1_index(size_t k, int j) {
    return ((k >> 3) * kHidden + (size_t)j) * 8 + (k & 1) * 4 + ((k & 7) >> 1);
}

// Number of windows of a launch: *n_dev (clamped to n_cap) when the count is
// held on the device, else n_cap.  Grids are sized for n_cap and loop.
__device__ inline int batch_n(const int* n_dev, int n_cap) {
    if (!n_dev) return n_cap;
    const int n = *n_dev;
    return n < n_cap ? n : n_cap;
}

// conv1: x [n][16][64] -> out [n][16][64][32]
// First convolution (1 -> 32 channels, 3x3, pad 1): one lane per output pixel
// loads the pixel's 3 x 3 neighbourhood once and computes all 32 channels,
// the weights and biases being wave-uniform values, then writes the pixel's
// 32 outputs (contiguous in NHWC) as 16-byte vectors.  Per channel the sum
// runs over (kh, kw) in order starting from the bias.
template <typename TO>
__device__ inline void conv1_pixel(const float* __restrict__ x, const float* __restrict__ w,
                                   const float* __restrict__ bias, TO* __restrict__ out, int64_t pix,
                                   float alpha) {
    const int col = (int)(pix % kGW);
    const int row = (int)((pix / kGW) % kGH);
    const int64_t n = pix / (kGW * kGH);
    const float* xi = x + n * kGH * kGW;
    float xv[9];
    bool ok[9];
#pragma unroll
    for (int kh = 0; kh < 3; ++kh)
#pragma unroll
        for (int kw = 0; kw < 3; ++kw) {
            const int r = row + kh - 1, q = col + kw - 1;
            const bool in = r >= 0 && r < kGH && q >= 0 && q < kGW;
            ok[kh * 3 + kw] = in;
            xv[kh * 3 + kw] = in ? xi[r * kGW + q] : 0.0f;
        }
    float acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = bias[c];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        if (!ok[t]) continue;
#pragma unroll
        for (int c = 0; c < 32; ++c) acc[c] = fmaf(w[t * 32 + c], xv[t], acc[c]);
    }
    TO* o = out + pix * 32;
    if constexpr (sizeof(TO) == 4) {
#pragma unroll
        for (int c = 0; c < 32; c += 4)
            *reinterpret_cast<float4*>(o + c) = make_float4(act_fn(acc[c], alpha), act_fn(acc[c + 1], alpha),
                                                            act_fn(acc[c + 2], alpha), act_fn(acc[c + 3], alpha));
    } else {
        typedef TO vec __attribute__((ext_vector_type(8)));
#pragma unroll
        for (int c = 0; c < 32; c += 8) {
            vec v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (TO)act_fn(acc[c + e], alpha);
            *reinterpret_cast<vec*>(o + c) = v;
        }
    }
}

__global__ __launch_bounds__(256) void k_conv1(const float* __restrict__ x, const float* __restrict__ w,
                                               const float* __restrict__ bias, float* __restrict__ out,
                                               const int* __restrict__ n_dev, int n_cap, float alpha) {
    const int64_t npix = (int64_t)batch_n(n_dev, n_cap) * kGH * kGW;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x)
        conv1_pixel<float>(x, w, bias, out, p, alpha);
}

// conv (Cin -> Cout), 3x3, pad 1, on MFMA f32 32x32x2.
// Workgroup: sample n, rows [h0, h0 + ROWS), ROWS = 64 / COUT; 4 waves, each a
// 32-pixel x 32-channel output block.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_mfma(const float* __restrict__ in,
                                                   const float* __restrict__ w,  // [9*CIN][COUT]
                                                   const float* __restrict__ bias,
                                                   float* __restrict__ out, const int* __restrict__ n_dev,
                                                   int n_cap, float alpha) {
    constexpr int ROWS = 64 / COUT;
    constexpr int PADW = kGW + 3;  // a zero column either side, odd stride
    constexpr int C4 = CIN / 4;
    constexpr int NCH = (ROWS + 2) * kGW * C4;   // 16-byte input chunks per block
    constexpr int PF = (NCH + 255) / 256;
    __shared__ float s_in[(ROWS + 2) * CIN * PADW];
    const int nblk = batch_n(n_dev, n_cap) * (kGH / ROWS);
    for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int n = blk / (kGH / ROWS);
        const int h0 = (blk % (kGH / ROWS)) * ROWS;
        const float* src = in + (size_t)n * kGH * kGW * CIN;
        // stage rows h0-1 .. h0+ROWS channel-major: every 16-byte load of the
        // block in flight at once, then the LDS stores
        float4 pf[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int c = threadIdx.x + 256 * q;
            pf[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (c < NCH) {
                const int r = c / (kGW * C4), col = (c / C4) % kGW, c4 = c % C4;
                const int gr = h0 - 1 + r;
                if (gr >= 0 && gr < kGH)
                    pf[q] = *reinterpret_cast<const float4*>(src + ((size_t)gr * kGW + col) * CIN + 4 * c4);
            }
        }
        for (int i = threadIdx.x; i < (ROWS + 2) * CIN * 2; i += 256)
            s_in[(i >> 1) * PADW + ((i & 1) ? kGW + 1 : 0)] = 0.0f;
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int c = threadIdx.x + 256 * q;
            if (c < NCH) {
                const int r = c / (kGW * C4), col = (c / C4) % kGW, c4 = c % C4;
                float* d = s_in + (r * CIN + 4 * c4) * PADW + col + 1;
                d[0] = pf[q].x;
                d[PADW] = pf[q].y;
                d[2 * PADW] = pf[q].z;
                d[3 * PADW] = pf[q].w;
            }
        }
        __syncthreads();
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        // block assignment: COUT = 64 -> (pixel half, cout half); COUT = 32 -> (row, pixel half)
        int rloc, px0, co0;
        if (COUT == 64) {
            rloc = 0;
            px0 = (wave & 1) * 32;
            co0 = (wave >> 1) * 32;
        } else {
            rloc = wave >> 1;
            px0 = (wave & 1) * 32;
            co0 = 0;
        }
        const int m = lane & 31, kk = lane >> 5;
        floatx16 acc = {};
#pragma unroll 1
        for (int kh = 0; kh < 3; ++kh) {
#pragma unroll 1
            for (int kw = 0; kw < 3; ++kw) {
                const float* arow = s_in + ((rloc + kh) * CIN) * PADW + px0 + m + kw;
                const float* wrow = w + (size_t)((kh * 3 + kw) * CIN) * COUT + co0 + m;
                // all CIN / 2 weight loads of this tap in flight before the products
                float bvs[CIN / 2];
#pragma unroll
                for (int c = 0; c < CIN; c += 2) bvs[c / 2] = wrow[(size_t)(c + kk) * COUT];
                __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the products
#pragma unroll
                for (int c = 0; c < CIN; c += 2)
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(arow[(c + kk) * PADW], bvs[c / 2], acc, 0, 0, 0);
            }
        }
        // D[i][j]: j = lane % 32 (output channel), i = 8 (v / 4) + 4 (lane / 32) + v % 4 (pixel)
        const int row = h0 + rloc;
        float* dst = out + ((size_t)n * kGH + row) * kGW * COUT;
        const float bj = bias[co0 + m];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int px = px0 + 8 * (v / 4) + 4 * kk + (v % 4);
            dst[(size_t)px * COUT + co0 + m] = act_fn(acc[v] + bj, alpha);
        }
        __syncthreads();   // s_in is restaged by the next iteration
    }
}

// Stages A[n0 .. n0 + 31][k0 .. k0 + kSplitK) (zero rows past n_total) into
// LDS rows of kSplitK + 1 floats (odd: the products' column reads are free of
// bank conflicts): all of the workgroup's 16-byte loads in flight, then the
// stores.
__device__ __forceinline__ void stage_rows(float* s_a, const float* __restrict__ a, int n0, int n_total, int k0) {
    constexpr int LDA = kSplitK + 1;
    constexpr int K4 = kSplitK / 4;
    constexpr int PF = 32 * K4 / 256;
    float4 pf[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int i = threadIdx.x + 256 * q;
        const int n = n0 + i / K4;
        pf[q] = n < n_total ? *reinterpret_cast<const float4*>(a + (size_t)n * kFlat + k0 + 4 * (i % K4))
                            : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int i = threadIdx.x + 256 * q;
        float* d = s_a + (i / K4) * LDA + 4 * (i % K4);
        d[0] = pf[q].x;
        d[1] = pf[q].y;
        d[2] = pf[q].z;
        d[3] = pf[q].w;
    }
}

// fc1 split-K: part[ks][row][128] = A[rows][kchunk] * W1[kchunk][128]
// grid (kNSplit, ceil(n / 32)); A = act (NHWC flatten, k = (h*64 + w)*64 + c).
__global__ __launch_bounds__(256) void k_fc1_mfma(const float* __restrict__ a, const float* __restrict__ w,
                                                  float* __restrict__ part, const int* __restrict__ n_dev,
                                                  int n_cap, int ld_part) {
    constexpr int LDA = kSplitK + 1;
    __shared__ float s_a[32 * LDA];
    const int n_total = batch_n(n_dev, n_cap);
    const int ks = blockIdx.x;
    const int k0 = ks * kSplitK;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, kk = lane >> 5;
    const int co0 = wave * 32;
    const float4* wp = reinterpret_cast<const float4*>(w) + ((size_t)(k0 >> 3) * kHidden + co0 + m) * 2 + kk;
    for (int mb = blockIdx.y; mb * 32 < n_total; mb += gridDim.y) {
        stage_rows(s_a, a, mb * 32, n_total, k0);
        __syncthreads();
        floatx16 acc = {};
#pragma unroll 1
        for (int g0 = 0; g0 < kSplitK / 8; g0 += 16) {   // 16 KB of weights in flight per wave
            float4 bvs[16];
#pragma unroll
            for (int g = 0; g < 16; ++g) bvs[g] = wp[(size_t)(g0 + g) * kHidden * 2];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                const float* ar = s_a + m * LDA + 8 * (g0 + g) + kk;
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[0], bvs[g].x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[2], bvs[g].y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[4], bvs[g].z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[6], bvs[g].w, acc, 0, 0, 0);
            }
        }
        float* dst = part + (size_t)ks * ld_part * kHidden;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = mb * 32 + 8 * (v / 4) + 4 * kk + (v % 4);
            dst[(size_t)r * kHidden + co0 + m] = acc[v];
        }
        __syncthreads();   // s_a is restaged by the next row block
    }
}

// fc1 for a batch whose count is held on the device (typically a few tens of
// windows) or of at most 64 windows: grid (kNSplit, 2), a workgroup per (K chunk, half of the 128
// outputs), so that twice as many workgroups stream the weights as with
// all 128 outputs per workgroup; wave (column block cb, K half kh) and the
// two K halves added in LDS in a fixed order.  Row blocks of 32 in a loop.
__global__ __launch_bounds__(256) void k_fc1_small(const float* __restrict__ a, const float* __restrict__ w,
                                                   float* __restrict__ part, const int* __restrict__ n_dev,
                                                   int n_cap, int ld_part) {
    constexpr int LDA = kSplitK + 1;
    constexpr int KH = kSplitK / 2;
    __shared__ float s_a[32 * LDA];
    __shared__ float s_red[2 * 16 * 64];
    const int n_total = batch_n(n_dev, n_cap);
    const int ks = blockIdx.x;
    const int k0 = ks * kSplitK;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, kk = lane >> 5;
    const int cb = wave & 1, kh = wave >> 1;
    const int co0 = blockIdx.y * 64 + cb * 32;
    const float4* wp = reinterpret_cast<const float4*>(w) + ((size_t)((k0 + kh * KH) >> 3) * kHidden + co0 + m) * 2 + kk;
    for (int mb = 0; mb * 32 < n_total; ++mb) {
        stage_rows(s_a, a, mb * 32, n_total, k0);
        __syncthreads();
        floatx16 acc = {};
#pragma unroll 1
        for (int g0 = 0; g0 < KH / 8; g0 += 16) {
            float4 bvs[16];
#pragma unroll
            for (int g = 0; g < 16; ++g) bvs[g] = wp[(size_t)(g0 + g) * kHidden * 2];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                const float* ar = s_a + m * LDA + kh * KH + 8 * (g0 + g) + kk;
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[0], bvs[g].x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[2], bvs[g].y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[4], bvs[g].z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[6], bvs[g].w, acc, 0, 0, 0);
            }
        }
        if (kh == 1) {
#pragma unroll
            for (int v = 0; v < 16; ++v) s_red[(cb * 16 + v) * 64 + lane] = acc[v];
        }
        __syncthreads();
        if (kh == 0) {
            float* dst = part + (size_t)ks * ld_part * kHidden;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = mb * 32 + 8 * (v / 4) + 4 * kk + (v % 4);
                dst[(size_t)r * kHidden + co0 + m] = acc[v] + s_red[(cb * 16 + v) * 64 + lane];
            }
        }
        __syncthreads();   // s_a and s_red are rewritten by the next row block
    }
}

// ---- 16-bit (bf16 / fp16) network: same layers, 16-bit operands, float32 accumulation
template <typename T> struct V8;
template <> struct V8<__bf16> { typedef bf16x8 type; };
template <> struct V8<_Float16> { typedef f16x8 type; };

template <typename T>
__device__ inline floatx16 mfma32(typename V8<T>::type a, typename V8<T>::type b, floatx16 c);
template <>
__device__ inline floatx16 mfma32<__bf16>(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
template <>
__device__ inline floatx16 mfma32<_Float16>(f16x8 a, f16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_conv1_16(const float* __restrict__ x, const float* __restrict__ w,
                                                  const float* __restrict__ bias, T* __restrict__ out,
                                                  const int* __restrict__ n_dev, int n_cap, float alpha) {
    const int64_t npix = (int64_t)batch_n(n_dev, n_cap) * kGH * kGW;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x)
        conv1_pixel<T>(x, w, bias, out, p, alpha);
}

// conv Cin -> Cout on v_mfma_f32_32x32x16_{bf16,f16} as an implicit GEMM with
// both operands staged in LDS.  A persistent 256-thread workgroup copies the
// layer's weights ([9][Cout][Cin], channel rows padded by 8 elements so that
// the 16-byte reads of 32 lanes spread over all banks) into LDS once, then
// loops over tiles of four output rows of one window: it stages the tile's
// six input rows (66 columns with the zero padding, NHWC, padded rows),
// issuing the next tile's global loads into registers before the products
// of this one.  Wave w computes output row w of the tile: 64 pixels x Cout
// channels as 2 x (Cout / 32) accumulators, one k step (16 channels of one
// kernel tap) reading one 16-byte weight fragment per 32 channels and one
// input fragment per 32 pixels.  The weights are the A operand (rows =
// output channels) and the inputs the B operand (columns = pixels), so each
// lane ends with four consecutive channels of one pixel per group and stores
// them as one 8-byte vector.
template <typename T, int CIN, int COUT>
struct Conv16Geo {
    static constexpr int CINP = CIN + 8;           // LDS channel stride (elements)
    static constexpr int ROWS = 4;                 // output rows per tile (one per wave)
    static constexpr int IR = ROWS + 2, IP = kGW + 2;
    static constexpr int W_ELEMS = 9 * COUT * CINP;
    static constexpr int I_ELEMS = IR * IP * CINP;
    static constexpr int CH = CIN / 8;             // 16-byte chunks per pixel
    static constexpr int IN_CHUNKS = IR * kGW * CH;
    static constexpr int PF = (IN_CHUNKS + 255) / 256;   // prefetched chunks per thread
};

template <typename T, int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv16_lds(const T* __restrict__ in, const T* __restrict__ w,
                                                    const float* __restrict__ bias, T* __restrict__ out,
                                                    const int* __restrict__ n_dev, int n_cap, float alpha) {
    typedef Conv16Geo<T, CIN, COUT> G;
    typedef typename V8<T>::type vec;
    typedef T vec4 __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) T s_w[G::W_ELEMS];
    __shared__ __attribute__((aligned(16))) T s_in[G::I_ELEMS];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 31, kg = lane >> 5;
    const int ntiles = batch_n(n_dev, n_cap) * (kGH / G::ROWS);
    if ((int)blockIdx.x >= ntiles) return;
    const vec zero = {};

    // weights, once per workgroup
    for (int c = tid; c < 9 * COUT * G::CH; c += 256) {
        const int row = c / G::CH, q = c % G::CH;   // row = kk * COUT + co
        *reinterpret_cast<vec*>(s_w + row * G::CINP + 8 * q) = *reinterpret_cast<const vec*>(w + (size_t)row * CIN + 8 * q);
    }
    // zero padding columns (pixel -1 and 64) of every staged row, never overwritten
    for (int c = tid; c < G::IR * 2 * G::CH; c += 256) {
        const int r = c / (2 * G::CH), side = (c / G::CH) & 1, q = c % G::CH;
        *reinterpret_cast<vec*>(s_in + (r * G::IP + (side ? G::IP - 1 : 0)) * G::CINP + 8 * q) = zero;
    }

    vec pf[G::PF];
    auto load_tile = [&](int tile) {
        const int n = tile / (kGH / G::ROWS);
        const int h0 = (tile % (kGH / G::ROWS)) * G::ROWS;
#pragma unroll
        for (int i = 0; i < G::PF; ++i) {
            const int c = tid + 256 * i;
            pf[i] = zero;
            if (c < G::IN_CHUNKS) {
                const int r = c / (kGW * G::CH), px = (c / G::CH) % kGW, q = c % G::CH;
                const int row = h0 - 1 + r;
                if (row >= 0 && row < kGH)
                    pf[i] = *reinterpret_cast<const vec*>(in + (((size_t)n * kGH + row) * kGW + px) * CIN + 8 * q);
            }
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int i = 0; i < G::PF; ++i) {
            const int c = tid + 256 * i;
            if (c < G::IN_CHUNKS) {
                const int r = c / (kGW * G::CH), px = (c / G::CH) % kGW, q = c % G::CH;
                *reinterpret_cast<vec*>(s_in + (r * G::IP + px + 1) * G::CINP + 8 * q) = pf[i];
            }
        }
    };

    constexpr int NCO = COUT / 32;
    int tile = blockIdx.x;
    load_tile(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        __syncthreads();   // the previous tile's products are done with s_in
        store_tile();
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) load_tile(tile + gridDim.x);   // in flight during the products
        floatx16 acc[NCO][2];
#pragma unroll
        for (int a = 0; a < NCO; ++a) acc[a][0] = acc[a][1] = floatx16{};
#pragma unroll
        for (int kh = 0; kh < 3; ++kh) {
#pragma unroll
            for (int kw = 0; kw < 3; ++kw) {
                const T* ip = s_in + ((wave + kh) * G::IP + m + kw) * G::CINP + 8 * kg;
                const T* wp = s_w + ((kh * 3 + kw) * COUT + m) * G::CINP + 8 * kg;
#pragma unroll
                for (int cb = 0; cb < CIN / 16; ++cb) {
                    vec bv[2], av[NCO];
#pragma unroll
                    for (int ph = 0; ph < 2; ++ph) bv[ph] = *reinterpret_cast<const vec*>(ip + ph * 32 * G::CINP + 16 * cb);
#pragma unroll
                    for (int a = 0; a < NCO; ++a) av[a] = *reinterpret_cast<const vec*>(wp + a * 32 * G::CINP + 16 * cb);
#pragma unroll
                    for (int a = 0; a < NCO; ++a)
#pragma unroll
                        for (int ph = 0; ph < 2; ++ph) acc[a][ph] = mfma32<T>(av[a], bv[ph], acc[a][ph]);
                }
            }
        }
        // lane: pixel ph * 32 + m; channels a * 32 + 8 g + 4 kg + (0..3)
        const int n = tile / (kGH / G::ROWS);
        const int row = (tile % (kGH / G::ROWS)) * G::ROWS + wave;
        T* dst = out + ((size_t)n * kGH + row) * kGW * COUT;
#pragma unroll
        for (int a = 0; a < NCO; ++a) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int co = a * 32 + 8 * g + 4 * kg;
                const float4 bb = *reinterpret_cast<const float4*>(bias + co);
#pragma unroll
                for (int ph = 0; ph < 2; ++ph) {
                    vec4 o;
                    o[0] = (T)act_fn(acc[a][ph][4 * g + 0] + bb.x, alpha);
                    o[1] = (T)act_fn(acc[a][ph][4 * g + 1] + bb.y, alpha);
                    o[2] = (T)act_fn(acc[a][ph][4 * g + 2] + bb.z, alpha);
                    o[3] = (T)act_fn(acc[a][ph][4 * g + 3] + bb.w, alpha);
                    *reinterpret_cast<vec4*>(dst + (size_t)(ph * 32 + m) * COUT + co) = o;
                }
            }
        }
    }
}

// fc1 split-K on 16-bit operands: A = act [n][65536] (NHWC flatten), B = W1 [128][65536].
template <typename T>
__global__ __launch_bounds__(256) void k_fc1_16(const T* __restrict__ a, const T* __restrict__ w,
                                                float* __restrict__ part, const int* __restrict__ n_dev,
                                                int n_cap, int ld_part) {
    typedef typename V8<T>::type vec;
    const int n_total = batch_n(n_dev, n_cap);
    const int ks = blockIdx.x;
    const int k0 = ks * kSplitK;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, kg = lane >> 5;
    const int co0 = wave * 32;
    const T* bp = w + (size_t)(co0 + m) * kFlat + k0 + kg * 8;
    for (int mb = blockIdx.y; mb * 32 < n_total; mb += gridDim.y) {
        const int n = mb * 32 + m;
        const bool valid = n < n_total;
        const T* ap = a + (size_t)(valid ? n : 0) * kFlat + k0 + kg * 8;
        floatx16 acc = {};
        vec zero = {};
#pragma unroll 1
        for (int k0 = 0; k0 < kSplitK; k0 += 8 * 16) {   // eight operand pairs in flight per group
            vec avs[8], bvs[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                avs[q] = valid ? *reinterpret_cast<const vec*>(ap + k0 + 16 * q) : zero;
                bvs[q] = *reinterpret_cast<const vec*>(bp + k0 + 16 * q);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 8; ++q) acc = mfma32<T>(avs[q], bvs[q], acc);
        }
        float* dst = part + (size_t)ks * ld_part * kHidden;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = mb * 32 + 8 * (v / 4) + 4 * kg + (v % 4);
            dst[(size_t)r * kHidden + co0 + m] = acc[v];
        }
    }
}

// fc1 on 16-bit operands for host-sized batches of at least 128 windows: a
// workgroup per (K chunk of kWideK, 128 windows), wave w owning windows
// 32 w .. 32 w + 31 and all 128 outputs (four accumulators), so each
// activation is read once from HBM and the weight fragments, common to the
// four waves, come from cache.  Workgroups of one K chunk are kSplitWide
// apart in launch order, which puts them on the same XCD (and L2).
constexpr int kWideK = 2048;
constexpr int kSplitWide = kFlat / kWideK;   // 32
template <typename T>
__global__ __launch_bounds__(256) void k_fc1_16w(const T* __restrict__ a, const T* __restrict__ w,
                                                 float* __restrict__ part, int n, int ld_part) {
    typedef typename V8<T>::type vec;
    constexpr int U = 4;   // k steps of 16 in flight
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, kg = lane >> 5;
    const int ks = blockIdx.x, k0 = ks * kWideK;
    const int row = blockIdx.y * 128 + wave * 32 + m;
    const bool valid = row < n;
    const T* ap = a + (size_t)(valid ? row : 0) * kFlat + k0 + kg * 8;
    const T* bp = w + (size_t)m * kFlat + k0 + kg * 8;
    const vec zero = {};
    floatx16 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = floatx16{};
#pragma unroll 1
    for (int k = 0; k < kWideK; k += 16 * U) {
        vec av[U], bv[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            av[u] = valid ? *reinterpret_cast<const vec*>(ap + k + 16 * u) : zero;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                bv[u][cb] = *reinterpret_cast<const vec*>(bp + (size_t)cb * 32 * kFlat + k + 16 * u);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma32<T>(av[u], bv[u][cb], acc[cb]);
    }
    float* dst = part + (size_t)ks * ld_part * kHidden;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int r = blockIdx.y * 128 + wave * 32 + 8 * (v / 4) + 4 * kg + (v % 4);
        if (r >= n) continue;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) dst[(size_t)r * kHidden + cb * 32 + m] = acc[cb][v];
    }
}

// float32 device layouts -> 16-bit copies: conv [(kh*3+kw)*Cin+cin][Cout] -> [kh*3+kw][Cout][Cin],
// fc1 [k][128] -> [128][k].
template <typename T>
__global__ void k_to16(const float* __restrict__ W, T* __restrict__ w16, ModelLayout lay, size_t o2, size_t o3,
                       size_t o4, size_t of1) {
    const size_t nth = (size_t)gridDim.x * blockDim.x;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    auto conv = [&](size_t src, size_t dst, int cin, int cout) {
        for (size_t i = tid; i < (size_t)9 * cin * cout; i += nth) {
            const int kk = (int)(i / ((size_t)cin * cout));
            const int ci = (int)((i / cout) % cin);
            const int co = (int)(i % cout);
            w16[dst + ((size_t)kk * cout + co) * cin + ci] = (T)W[src + i];
        }
    };
    conv(lay.w2, o2, 32, 32);
    conv(lay.w3, o3, 32, 64);
    conv(lay.w4, o4, 64, 64);
    for (size_t i = tid; i < (size_t)kFlat * kHidden; i += nth) {
        const size_t k = i / kHidden;
        const int j = (int)(i % kHidden);
        w16[of1 + (size_t)j * kFlat + k] = (T)W[lay.f1 + f1_index(k, j)];
    }
}

__device__ inline float softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }

// fc1's reduction, fc2 and the head, one sample per 1024-thread workgroup
// (samples in a loop): thread (g, j) sums the partials ks = g, g + 8, ...
// (nsplit K chunks, a multiple of 8)
// of hidden unit j in order, the eight group sums are added in order (then
// the bias and phi), and wave o < 14 forms output o from the 128 hidden
// values (two per lane, lanes combined by a fixed butterfly), so the result
// does not depend on the launch.  mu = out[0:4]; L = out[4:14] with
// softplus on the diagonal entries (packed positions 0, 2, 5, 9).
__global__ __launch_bounds__(1024) void k_fc1_head(const float* __restrict__ part, const float* __restrict__ b1,
                                                   const float* __restrict__ w2,   // [14][128]
                                                   const float* __restrict__ b2, float* __restrict__ mu,
                                                   float* __restrict__ L, const int* __restrict__ n_dev, int n_cap,
                                                   int ld_part, int nsplit, float alpha) {
    constexpr int G = 8;
    __shared__ float s_p[G * kHidden];
    __shared__ float s_h[kHidden];
    const int tid = threadIdx.x;
    const int j = tid & (kHidden - 1), g = tid >> 7;
    const int wave = tid >> 6, lane = tid & 63;
    const int n_total = batch_n(n_dev, n_cap);
    for (int n = blockIdx.x; n < n_total; n += gridDim.x) {
        float acc = 0.0f;
#pragma unroll
        for (int ks = g; ks < nsplit; ks += G) acc += part[((size_t)ks * ld_part + n) * kHidden + j];
        s_p[g * kHidden + j] = acc;
        __syncthreads();
        if (tid < kHidden) {
            float h = 0.0f;
#pragma unroll
            for (int q = 0; q < G; ++q) h += s_p[q * kHidden + tid];
            s_h[tid] = act_fn(h + b1[tid], alpha);
        }
        __syncthreads();
        if (wave < kOut) {
            const float* wr = w2 + (size_t)wave * kHidden;
            float v = fmaf(wr[lane], s_h[lane], wr[lane + 64] * s_h[lane + 64]);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) {
                v += b2[wave];
                if (wave < 4) {
                    mu[(size_t)n * 4 + wave] = v;
                } else {
                    const int p = wave - 4;
                    const bool diag = p == 0 || p == 2 || p == 5 || p == 9;
                    L[(size_t)n * 10 + p] = diag ? softplus(v) : v;
                }
            }
        }
        __syncthreads();   // s_p and s_h are rewritten for the next sample
    }
}

// Re-layout of the host blob (PyTorch layouts) into the device layouts.
__global__ void k_relayout(const float* __restrict__ blob, float* __restrict__ dst, ModelLayout lay) {
    // blob offsets (PyTorch order)
    const size_t o_w1 = 0, o_b1 = o_w1 + 32 * 9, o_w2 = o_b1 + 32, o_b2 = o_w2 + 32 * 32 * 9,
                 o_w3 = o_b2 + 32, o_b3 = o_w3 + 64 * 32 * 9, o_w4 = o_b3 + 64, o_b4 = o_w4 + 64 * 64 * 9,
                 o_f1 = o_b4 + 64, o_fb1 = o_f1 + (size_t)kHidden * kFlat, o_f2 = o_fb1 + kHidden,
                 o_fb2 = o_f2 + kOut * kHidden;
    const size_t nthreads = (size_t)gridDim.x * blockDim.x;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    // conv1: [32][1][3][3] -> [9][32]
    for (size_t i = tid; i < 32 * 9; i += nthreads) {
        const int c = (int)(i / 9), k = (int)(i % 9);
        dst[lay.w1 + k * 32 + c] = blob[o_w1 + i];
    }
    for (size_t i = tid; i < 32; i += nthreads) dst[lay.b1 + i] = blob[o_b1 + i];
    // conv2..4: [Cout][Cin][3][3] -> [(kh*3+kw)*Cin + cin][Cout]
    auto conv = [&](size_t ob, size_t od, int cin, int cout) {
        for (size_t i = tid; i < (size_t)cout * cin * 9; i += nthreads) {
            const int co = (int)(i / (cin * 9));
            const int ci = (int)((i / 9) % cin);
            const int k = (int)(i % 9);
            dst[od + ((size_t)k * cin + ci) * cout + co] = blob[ob + i];
        }
    };
    conv(o_w2, lay.w2, 32, 32);
    conv(o_w3, lay.w3, 32, 64);
    conv(o_w4, lay.w4, 64, 64);
    for (size_t i = tid; i < 32; i += nthreads) dst[lay.b2 + i] = blob[o_b2 + i];
    for (size_t i = tid; i < 64; i += nthreads) dst[lay.b3 + i] = blob[o_b3 + i];
    for (size_t i = tid; i < 64; i += nthreads) dst[lay.b4 + i] = blob[o_b4 + i];
    // fc1: [128][c*1024 + h*64 + w] -> [(h*64 + w)*64 + c][128]
    for (size_t i = tid; i < (size_t)kHidden * kFlat; i += nthreads) {
        const int j = (int)(i / kFlat);
        const int kt = (int)(i % kFlat);
        const int c = kt / (kGH * kGW), hw = kt % (kGH * kGW);
        dst[lay.f1 + f1_index((size_t)hw * 64 + c, j)] = blob[o_f1 + i];
    }
    for (size_t i = tid; i < kHidden; i += nthreads) dst[lay.fb1 + i] = blob[o_fb1 + i];
    for (size_t i = tid; i < (size_t)kOut * kHidden; i += nthreads) dst[lay.f2 + i] = blob[o_f2 + i];
    for (size_t i = tid; i < kOut; i += nthreads) dst[lay.fb2 + i] = blob[o_fb2 + i];
}

size_t blob_floats() {
    return 32 * 9 + 32 + 32 * 32 * 9 + 32 + 64 * 32 * 9 + 64 + 64 * 64 * 9 + 64 + (size_t)kHidden * kFlat +
           kHidden + kOut * kHidden + kOut;
}

int pad32(int n) { return (n + 31) / 32 * 32; }

// Result block: hdr[4] int32, rows[maxb][2] int32, mu[maxb][4], L[maxb][10] float32.
size_t out_block_bytes(int maxb) { return (4 + (size_t)maxb * (2 + 4 + 10)) * 4; }

size_t work_bytes(int precision, int maxb) {
    const size_t elt = precision == LPF_PREC_FP32 ? sizeof(float) : 2;
    const size_t act = (size_t)maxb * kGH * kGW * 64 * elt;
    size_t b = 0;
    b += 2 * align64(act);
    if (precision != LPF_PREC_FP32) b += align64(kW16total * 2);
    b += align64((size_t)kNSplit * pad32(maxb) * kHidden * sizeof(float));
    b += (1 + kInflight) * align64((size_t)maxb * kGH * kGW * sizeof(float));
    b += (1 + kInflight) * align64(out_block_bytes(maxb));
    return b;
}

}  // namespace

// Grid sizes for n_cap windows; with the count on the device the grids loop.
inline int grid_cap(int64_t want, int cap) { return (int)(want < 1 ? 1 : (want > cap ? cap : want)); }

// Grid caps: with the count held on the device most of an n_cap-sized grid
// would exit at once (and hold LDS while being dispatched), so those launches
// use about one workgroup per CU and loop; the network then takes fewer CUs
// from the filters and the catalogue it runs beside (measured: step 0.319 ms
// with 512-workgroup convolutions, 0.315 with 256, 0.335 with 128).
struct GridCaps {
    int conv1, conv, fc1_rows, head;
    explicit GridCaps(const int* n_dev)
        : conv1(n_dev ? 256 : 4096), conv(n_dev ? 256 : 2048), fc1_rows(n_dev ? 2 : 4), head(n_dev ? 256 : 1024) {}
};

// Device buffers one forward pass writes besides its outputs: two activation
// planes and the fc1 split-K partials (leading dimension ldp rows).  A
// model's own workspace provides them, or the library's static scratch
// array (lpf_infer_windows_static).
struct NetBufs {
    void* act_a;
    void* act_b;
    float* part;
    int ldp;
};

NetBufs model_bufs(const lpf_model* m) {
    const CnnWork& w = m->work;
    NetBufs nb;
    nb.act_a = m->precision == LPF_PREC_FP32 ? static_cast<void*>(w.act_a) : w.act16_a;
    nb.act_b = m->precision == LPF_PREC_FP32 ? static_cast<void*>(w.act_b) : w.act16_b;
    nb.part = w.part;
    nb.ldp = pad32(m->max_batch);
    return nb;
}

template <typename T>
hipError_t forward16(const lpf_model* m, const NetBufs& nb, const float* windows, const int* n_dev, int n_cap,
                     hipStream_t s, int* nsplit) {
    const ModelLayout& lay = m->lay;
    const float* W = m->wts;
    const T* w16 = static_cast<const T*>(m->work.w16);
    T* a = static_cast<T*>(nb.act_a);
    T* b = static_cast<T*>(nb.act_b);
    const GridCaps gc(n_dev);
    hipLaunchKernelGGL((k_conv1_16<T>), dim3(grid_cap(((int64_t)n_cap * kGH * kGW + 255) / 256, gc.conv1)),
                       dim3(256), 0, s, windows, W + lay.w1, W + lay.b1, a, n_dev, n_cap, m->alpha);
    // persistent implicit GEMMs: a workgroup per CU (Cin = 64: 137 KB of LDS) or two
    const int64_t tiles = (int64_t)n_cap * (kGH / 4);
    hipLaunchKernelGGL((k_conv16_lds<T, 32, 32>), dim3(grid_cap(tiles, 512)), dim3(256), 0, s, a, w16 + kW16o2,
                       W + lay.b2, b, n_dev, n_cap, m->alpha);
    hipLaunchKernelGGL((k_conv16_lds<T, 32, 64>), dim3(grid_cap(tiles, 512)), dim3(256), 0, s, b, w16 + kW16o3,
                       W + lay.b3, a, n_dev, n_cap, m->alpha);
    hipLaunchKernelGGL((k_conv16_lds<T, 64, 64>), dim3(grid_cap(tiles, 256)), dim3(256), 0, s, a, w16 + kW16o4,
                       W + lay.b4, b, n_dev, n_cap, m->alpha);
    // fc1: no LDS, so a host-sized batch gets a workgroup per (K chunk, 32 windows) to keep
    // enough loads in flight to stream the activations
    if (!n_dev && n_cap >= 128) {
        hipLaunchKernelGGL((k_fc1_16w<T>), dim3(kSplitWide, (n_cap + 127) / 128), dim3(256), 0, s, b, w16 + kW16of1,
                           nb.part, n_cap, nb.ldp);
        *nsplit = kSplitWide;
    } else {
        hipLaunchKernelGGL((k_fc1_16<T>), dim3(kNSplit, grid_cap((n_cap + 31) / 32, n_dev ? gc.fc1_rows : 32)),
                           dim3(256), 0, s, b, w16 + kW16of1, nb.part, n_dev, n_cap, nb.ldp);
        *nsplit = kNSplit;
    }
    return hipGetLastError();
}

// Runs the network on the device windows [0, n) with n = *n_dev clamped to
// n_cap when n_dev is given, else n = n_cap (n_cap <= the rows nb holds).
hipError_t forward_on(const lpf_model* m, const NetBufs& nb, const float* windows, const int* n_dev, int n_cap,
                      float* mu, float* L, hipStream_t s) {
    if (n_cap <= 0) return hipSuccess;
    const ModelLayout& lay = m->lay;
    const float* W = m->wts;
    const GridCaps gc(n_dev);
    hipError_t e = hipSuccess;
    int nsplit = kNSplit;
    if (m->precision == LPF_PREC_BF16) {
        e = forward16<__bf16>(m, nb, windows, n_dev, n_cap, s, &nsplit);
    } else if (m->precision == LPF_PREC_FP16) {
        e = forward16<_Float16>(m, nb, windows, n_dev, n_cap, s, &nsplit);
    } else {
        float* a = static_cast<float*>(nb.act_a);
        float* b = static_cast<float*>(nb.act_b);
        hipLaunchKernelGGL(k_conv1, dim3(grid_cap(((int64_t)n_cap * kGH * kGW + 255) / 256, gc.conv1)),
                           dim3(256), 0, s, windows, W + lay.w1, W + lay.b1, a, n_dev, n_cap, m->alpha);
        hipLaunchKernelGGL((k_conv_mfma<32, 32>), dim3(grid_cap((int64_t)n_cap * (kGH / 2), gc.conv)), dim3(256),
                           0, s, a, W + lay.w2, W + lay.b2, b, n_dev, n_cap, m->alpha);
        hipLaunchKernelGGL((k_conv_mfma<32, 64>), dim3(grid_cap((int64_t)n_cap * kGH, gc.conv)), dim3(256), 0, s,
                           b, W + lay.w3, W + lay.b3, a, n_dev, n_cap, m->alpha);
        hipLaunchKernelGGL((k_conv_mfma<64, 64>), dim3(grid_cap((int64_t)n_cap * kGH, gc.conv)), dim3(256), 0, s,
                           a, W + lay.w4, W + lay.b4, b, n_dev, n_cap, m->alpha);
        if (n_dev || n_cap <= 64)
            hipLaunchKernelGGL(k_fc1_small, dim3(kNSplit, 2), dim3(256), 0, s, b, W + lay.f1, nb.part, n_dev, n_cap,
                               nb.ldp);
        else
            hipLaunchKernelGGL(k_fc1_mfma, dim3(kNSplit, grid_cap((n_cap + 31) / 32, gc.fc1_rows)), dim3(256), 0, s,
                               b, W + lay.f1, nb.part, n_dev, n_cap, nb.ldp);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fc1_head, dim3(grid_cap(n_cap, gc.head)), dim3(1024), 0, s, nb.part, W + lay.fb1,
                       W + lay.f2, W + lay.fb2, mu, L, n_dev, n_cap, nb.ldp, nsplit, m->alpha);
    return hipGetLastError();
}

hipError_t cnn_forward(const lpf_model* m, const float* windows, const int* n_dev, int n_cap, float* mu,
                       float* L, hipStream_t s) {
    return forward_on(m, model_bufs(m), windows, n_dev, n_cap, mu, L, s);
}

// ---- allocation-free inference: a file-scope device scratch array --------
// Holds the buffers of one forward pass of up to kStaticWindows windows:
// two float32 activation planes and the fc1 partials (32 rows).  Each device has its own copy; host code reaches it only through
// the address hipGetSymbolAddress returns on that device.
constexpr int kStaticWindows = 32;
constexpr size_t kStaticAct = (size_t)kStaticWindows * kGH * kGW * 64 * sizeof(float);   // 8 MiB
constexpr size_t kStaticPart = (size_t)kNSplit * kStaticWindows * kHidden * sizeof(float);  // 2 MiB
constexpr size_t kStaticBytes = 2 * kStaticAct + kStaticPart;
static_assert(kStaticAct % 256 == 0 && kStaticPart % 256 == 0, "scratch sub-buffer alignment");

__device__ __align__(256) char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// (with that device current) and kept.
hipError_t scratch_address(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int static_max_windows() { return kStaticWindows; }
size_t static_scratch_bytes() { return kStaticBytes; }

// The network on n <= kStaticWindows device windows with the scratch array
// as its buffers, on stream s; no allocation of any kind.
hipError_t cnn_forward_static(const lpf_model* m, const float* windows, int n, float* mu, float* L, hipStream_t s) {
    char* base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return e;
    NetBufs nb;
    nb.act_a = base;
    nb.act_b = base + kStaticAct;
    nb.part = reinterpret_cast<float*>(base + 2 * kStaticAct);
    nb.ldp = kStaticWindows;
    return forward_on(m, nb, windows, nullptr, n, mu, L, s);
}

float* model_window_buffer(const lpf_model* m) { return m->work.windows; }
float* model_mu_buffer(const lpf_model* m) { return m->work.mu; }
float* model_L_buffer(const lpf_model* m) { return m->work.L; }
int model_max_batch(const lpf_model* m) { return m->max_batch; }

// Pinned host rows of 14 floats (mu then L) for n results; grows by doubling.
float* model_host_rows(const lpf_model* m, size_t n) {
    if (n > m->h_cap) {
        size_t cap = m->h_cap ? m->h_cap : 256;
        while (cap < n) cap *= 2;
        float* p = nullptr;
        if (hipHostMalloc(reinterpret_cast<void**>(&p), cap * 14 * sizeof(float), hipHostMallocDefault) !=
            hipSuccess)
            return nullptr;
        if (m->h_out) (void)hipHostFree(m->h_out);
        m->h_out = p;
        m->h_cap = cap;
    }
    return m->h_out;
}

size_t model_blob_bytes() { return (blob_floats() + 1) * sizeof(float); }

int model_workspace_size(int precision, int maxb, size_t* bytes) {
    if (precision != LPF_PREC_FP32 && precision != LPF_PREC_BF16 && precision != LPF_PREC_FP16)
        return LPF_EINVAL;
    if (maxb < 1 || maxb > 65536) return LPF_EINVAL;
    *bytes = align64(make_layout().total * sizeof(float)) + work_bytes(precision, maxb) +
             align64(blob_floats() * sizeof(float));
    return LPF_OK;
}

void model_destroy(lpf_model* m);

int model_create(const void* weights, size_t bytes, int precision, int maxb, void* ws, size_t ws_bytes,
                 hipStream_t s, lpf_model** out) {
    if (!weights || !ws || !out) return LPF_EINVAL;
    if (bytes != model_blob_bytes()) return LPF_EINVAL;
    size_t need;
    int rc = model_workspace_size(precision, maxb, &need);
    if (rc != LPF_OK) return rc;
    if (ws_bytes < need) return LPF_ENOMEM;
    lpf_model* m = new lpf_model();
    m->precision = precision;
    m->max_batch = maxb;
    m->lay = make_layout();
    m->stream = s;
    const float* hb = static_cast<const float*>(weights);
    m->alpha = hb[blob_floats()];
    char* p = static_cast<char*>(ws);
    m->wts = reinterpret_cast<float*>(p);
    p += align64(m->lay.total * sizeof(float));
    const size_t elt = precision == LPF_PREC_FP32 ? sizeof(float) : 2;
    const size_t act = align64((size_t)maxb * kGH * kGW * 64 * elt);
    m->work.act_a = nullptr;
    m->work.act_b = nullptr;
    m->work.act16_a = nullptr;
    m->work.act16_b = nullptr;
    m->work.w16 = nullptr;
    if (precision == LPF_PREC_FP32) {
        m->work.act_a = reinterpret_cast<float*>(p); p += act;
        m->work.act_b = reinterpret_cast<float*>(p); p += act;
    } else {
        m->work.act16_a = p; p += act;
        m->work.act16_b = p; p += act;
        m->work.w16 = p; p += align64(kW16total * 2);
    }
    m->work.part = reinterpret_cast<float*>(p);
    p += align64((size_t)kNSplit * pad32(maxb) * kHidden * sizeof(float));
    m->work.windows = reinterpret_cast<float*>(p); p += align64((size_t)maxb * kGH * kGW * sizeof(float));
    m->work.hdr = reinterpret_cast<int32_t*>(p);
    m->work.rows = m->work.hdr + 4;
    m->work.mu = reinterpret_cast<float*>(m->work.rows + 2 * (size_t)maxb);
    m->work.L = m->work.mu + 4 * (size_t)maxb;
    m->work.out_bytes = out_block_bytes(maxb);
    p += align64(m->work.out_bytes);
    for (int i = 0; i < kInflight; ++i) {
        m->work.swin[i] = reinterpret_cast<float*>(p); p += align64((size_t)maxb * kGH * kGW * sizeof(float));
        m->work.sblk[i] = reinterpret_cast<int32_t*>(p); p += align64(m->work.out_bytes);
    }
    float* staging = reinterpret_cast<float*>(p);
    hipError_t e = hipMemcpyAsync(staging, weights, blob_floats() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_relayout, dim3(1024), dim3(256), 0, s, staging, m->wts, m->lay);
        e = hipGetLastError();
    }
    if (e == hipSuccess && precision == LPF_PREC_BF16) {
        hipLaunchKernelGGL((k_to16<__bf16>), dim3(1024), dim3(256), 0, s, m->wts,
                           static_cast<__bf16*>(m->work.w16), m->lay, kW16o2, kW16o3, kW16o4, kW16of1);
        e = hipGetLastError();
    } else if (e == hipSuccess && precision == LPF_PREC_FP16) {
        hipLaunchKernelGGL((k_to16<_Float16>), dim3(1024), dim3(256), 0, s, m->wts,
                           static_cast<_Float16*>(m->work.w16), m->lay, kW16o2, kW16o3, kW16o4, kW16of1);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // inference stream (default priority), events and pinned result blocks;
    // the events that order kernels after kernels of this device skip the
    // system-scope fence; ev_in / ev_out (the caller's stream, which may carry
    // copies) and ev_done (waited on by the host) keep it
    constexpr unsigned kDevEvent = hipEventDisableTiming | hipEventDisableSystemFence;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->istream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_gathered, kDevEvent);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming);
    for (int i = 0; i < kInflight && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&m->ev_done[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_gath[i], kDevEvent);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&m->h_res[i]), m->work.out_bytes, hipHostMallocDefault);
    }
    if (e != hipSuccess) {
        model_destroy(m);
        return LPF_EDEVICE;
    }
    *out = m;
    return LPF_OK;
}

void model_destroy(lpf_model* m) {
    if (!m) return;
    if (m->istream) (void)hipStreamSynchronize(m->istream);
    for (int i = 0; i < kInflight; ++i) {
        if (m->pend_ctx[i]) {   // a deferred launch that will not happen: its ticket dies with the model
            // its gather (on the context's stream) still writes this model's buffers
            (void)hipStreamSynchronize(m->pend_ctx[i]->stream);
            m->pend_ctx[i]->pend_model = nullptr;
            m->pend_ctx[i]->pend_slot = -1;
        }
        if (m->ev_done[i]) (void)hipEventDestroy(m->ev_done[i]);
        if (m->ev_gath[i]) (void)hipEventDestroy(m->ev_gath[i]);
        if (m->h_res[i]) (void)hipHostFree(m->h_res[i]);
    }
    if (m->ev_gathered) (void)hipEventDestroy(m->ev_gathered);
    if (m->ev_in) (void)hipEventDestroy(m->ev_in);
    if (m->ev_out) (void)hipEventDestroy(m->ev_out);
    if (m->istream) (void)hipStreamDestroy(m->istream);
    if (m->h_out) (void)hipHostFree(m->h_out);
    delete m;
}

}  // namespace lpf
