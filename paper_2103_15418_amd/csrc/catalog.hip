// Source association and monitoring (Sec. 2.2), one workgroup per step.
//
// Input: the per-band peak lists written by the detection pass.  Steps:
//  0. release records reported as ended at the previous step; end episodes
//     a gap in t carried past their last measured step;
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

struct CatArgs {
    int B, peak_cap, max_sources, n_mon;
    float r_dup2, r_assoc2;
    int64_t t;
    const int32_t* peak_cnt;
    const PeakRec* peak_raw;
    PeakRec* peak_sorted;
    int32_t* order;     // [kCatMaxPeaks] bij-rank by visiting position
    int32_t* nbr;       // [kCatMaxPeaks][kNbr + 1]
    int32_t* cand;      // [kCatMaxPeaks][kCand + 1]
    int32_t* kept;      // [kCatMaxPeaks] kept peaks (bij rank) in visiting order
    int32_t* free_list; // [max_sources]
    int32_t* src_id;
    int32_t* src_row;
    int32_t* src_col;
    int32_t* src_state;
    int64_t* src_tfirst;
    int64_t* src_tlast;
    int64_t* src_tend;
    int32_t* src_new;
    int32_t* list_measured;
    int32_t* list_new;
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

__device__ inline int pack_pos(int i, int j) { return (i << 16) | j; }
__device__ inline int pos_i(int p) { return p >> 16; }
__device__ inline int pos_j(int p) { return p & 0xffff; }
__device__ inline float dist2(int a, int b) {
    const float di = (float)(pos_i(a) - pos_i(b)), dj = (float)(pos_j(a) - pos_j(b));
    return di * di + dj * dj;
}

__global__ __launch_bounds__(kCatThreads) void k_catalog(CatArgs a) {
    __shared__ uint64_t s_keys[kCatMaxPeaks];        // 64 KB: sort keys, later live lists
    __shared__ int32_t s_pos[kCatMaxPeaks];          // 32 KB: positions in visiting order
    __shared__ uint8_t s_flag[kCatMaxPeaks];         //  8 KB: kept flags
    __shared__ uint32_t s_taken[kMaxSources / 32];   //  8 KB: taken bitmap
    __shared__ int s_off[kMaxB + 1];
    __shared__ int s_tmp[kCatThreads / 64 + 1];
    __shared__ int s_P, s_K, s_nlive, s_held, s_nfree, s_nnew, s_drop, s_next;
    __shared__ uint32_t s_overflow;

    const int tid = threadIdx.x;
    const int S = a.max_sources;
    const int64_t t = a.t;

    // ---- 0. release previous ended records; end episodes left over by a gap
    for (int s = tid; s < S; s += kCatThreads) {
        int st = a.src_state[s];
        if (st == kSrcEnded) {
            st = kSrcFree;
        } else if (st == kSrcLive && t - a.src_tlast[s] > a.n_mon) {
            st = kSrcEnded;
            a.src_tend[s] = a.src_tlast[s] + a.n_mon;
        }
        a.src_state[s] = st;
        a.src_new[s] = 0;
    }
    for (int w = tid; w < (S + 31) / 32; w += kCatThreads) s_taken[w] = 0u;
    if (tid == 0) {
        int off = 0;
        uint32_t ovf = 0;
        for (int b = 0; b < a.B; ++b) {
            const int n = a.peak_cnt[b];
            s_off[b] = off;
            if (n > a.peak_cap) ovf |= 1u << b;
            else off += n;
        }
        s_off[a.B] = off;
        s_P = off;
        s_overflow = ovf;
        s_next = a.status->next_id;
    }
    __syncthreads();
    const int P = s_P;

    // ---- 1. (band, row, col) order
    int Ppad = 1;
    while (Ppad < P) Ppad <<= 1;
    for (int n = tid; n < Ppad; n += kCatThreads) s_keys[n] = ~0ull;
    __syncthreads();
    for (int b = 0; b < a.B; ++b) {
        if ((s_overflow >> b) & 1u) continue;
        const int n0 = s_off[b], cnt = s_off[b + 1] - n0;
        for (int q = tid; q < cnt; q += kCatThreads) {
            const PeakRec& r = a.peak_raw[(size_t)b * a.peak_cap + q];
            const uint32_t key = ((uint32_t)r.band << 24) | ((uint32_t)r.row << 12) | (uint32_t)r.col;
            s_keys[n0 + q] = ((uint64_t)key << 32) | (uint32_t)(b * a.peak_cap + q);
        }
    }
    __syncthreads();
    if (P > 1) bitonic_sort(s_keys, Ppad);
    for (int n = tid; n < P; n += kCatThreads) {
        const uint32_t ref = (uint32_t)(s_keys[n] & 0xffffffffu);
        a.peak_sorted[n] = a.peak_raw[ref];
    }
    __syncthreads();  // peak_sorted is read back below (global, same block)

    // ---- 2. visiting order: x descending, then (band, row, col) = rank
    for (int n = tid; n < Ppad; n += kCatThreads) {
        if (n < P) {
            const uint32_t ox = ~ordered(a.peak_sorted[n].x);
            s_keys[n] = ((uint64_t)ox << 32) | (uint32_t)n;
        } else {
            s_keys[n] = ~0ull;
        }
    }
    __syncthreads();
    if (P > 1) bitonic_sort(s_keys, Ppad);
    for (int q = tid; q < P; q += kCatThreads) {
        const int n = (int)(s_keys[q] & 0xffffffffu);
        a.order[q] = n;
        s_pos[q] = pack_pos(a.peak_sorted[n].row, a.peak_sorted[n].col);
    }
    __syncthreads();

    // ---- 3. duplicate removal: neighbour lists, then greedy resolution.
    // nbr[q] = {count, up to kNbr earlier-visited peaks within dup_radius}.
    for (int q = tid; q < P; q += kCatThreads) {
        const int pq = s_pos[q];
        int32_t* nb = a.nbr + (size_t)q * (kNbr + 1);
        int cnt = 0;
        for (int r = 0; r < q; ++r) {
            if (dist2(pq, s_pos[r]) <= a.r_dup2) {
                if (cnt < kNbr) nb[1 + cnt] = r;
                ++cnt;
            }
        }
        nb[0] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        int K = 0;
        for (int q = 0; q < P; ++q) {
            const int32_t* nb = a.nbr + (size_t)q * (kNbr + 1);
            const int cnt = nb[0];
            bool keep = true;
            if (cnt > kNbr) {  // long list: test against every kept peak so far
                for (int r = 0; r < K && keep; ++r)
                    if (dist2(s_pos[q], s_pos[a.kept[r]]) <= a.r_dup2) keep = false;
            } else {
                for (int r = 0; r < cnt && keep; ++r)
                    if (s_flag[nb[1 + r]]) keep = false;
            }
            s_flag[q] = keep ? 1 : 0;
            if (keep) a.kept[K++] = q;
        }
        s_K = K;
    }
    __syncthreads();
    const int K = s_K;

    // ---- 4a. live sources (compacted, slot order) and the free list
    int32_t* s_live = reinterpret_cast<int32_t*>(s_keys);        // [S <= 8192 fast path]
    int32_t* s_lpos = s_live + kCatMaxPeaks;
    {
        const int per = (S + kCatThreads - 1) / kCatThreads;
        const int s0 = tid * per, s1 = min(S, s0 + per);
        int nl = 0, nf = 0, nh = 0;
        for (int s = s0; s < s1; ++s) {
            const int st = a.src_state[s];
            nl += st == kSrcLive;
            nf += st == kSrcFree;
            nh += st != kSrcFree;
        }
        int tot;
        int ol = block_scan(nl, s_tmp, &tot);
        if (tid == 0) s_nlive = tot;
        int of = block_scan(nf, s_tmp, &tot);
        if (tid == 0) s_nfree = tot;
        int oh = block_scan(nh, s_tmp, &tot);
        (void)oh;
        if (tid == 0) s_held = tot;
        for (int s = s0; s < s1; ++s) {
            const int st = a.src_state[s];
            if (st == kSrcLive) {
                if (ol < kCatMaxPeaks) {
                    s_live[ol] = s;
                    s_lpos[ol] = pack_pos(a.src_row[s], a.src_col[s]);
                }
                ++ol;
            } else if (st == kSrcFree) {
                a.free_list[of++] = s;
            }
        }
    }
    __syncthreads();
    const int L = s_nlive;
    const bool live_in_lds = L <= kCatMaxPeaks;

    // ---- 4b. association candidates of each kept peak, sorted by (d^2, id).
    // cand[kq] = {count or -1 (too many / table not staged), up to kCand slots}.
    for (int kq = tid; kq < K; kq += kCatThreads) {
        int32_t* out = a.cand + (size_t)kq * (kCand + 1);
        if (!live_in_lds) {
            out[0] = -1;
            continue;
        }
        const int pq = s_pos[a.kept[kq]];
        float cd[kCand];
        int cid[kCand], cs[kCand];
        int cnt = 0;
        for (int l = 0; l < L; ++l) {
            const float d = dist2(pq, s_lpos[l]);
            if (d > a.r_assoc2) continue;
            if (cnt == kCand) {
                cnt = kCand + 1;
                break;
            }
            const int s = s_live[l];
            const int id = a.src_id[s];
            int m = cnt++;
            while (m > 0 && (cd[m - 1] > d || (cd[m - 1] == d && cid[m - 1] > id))) {
                cd[m] = cd[m - 1];
                cid[m] = cid[m - 1];
                cs[m] = cs[m - 1];
                --m;
            }
            cd[m] = d;
            cid[m] = id;
            cs[m] = s;
        }
        if (cnt > kCand) {
            out[0] = -1;
        } else {
            out[0] = cnt;
            for (int m = 0; m < cnt; ++m) out[1 + m] = cs[m];
        }
    }
    __syncthreads();

    // ---- 4c. greedy resolution (visiting order)
    if (tid == 0) {
        int held = s_held, nnew = 0, drop = 0, next = s_next;
        for (int kq = 0; kq < K; ++kq) {
            const int32_t* cl = a.cand + (size_t)kq * (kCand + 1);
            int match = -1;
            if (cl[0] < 0) {
                // exact scan of the whole table (sources opened this step are taken)
                const int pq = s_pos[a.kept[kq]];
                float bd = 0.0f;
                int bid = 0;
                for (int s = 0; s < S; ++s) {
                    if (a.src_state[s] != kSrcLive) continue;
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
                a.src_tlast[match] = t;
                continue;
            }
            if (held >= S || nnew >= s_nfree) {
                ++drop;
                continue;
            }
            const int s = a.free_list[nnew++];
            ++held;
            const int n = a.order[a.kept[kq]];
            a.src_id[s] = next++;
            a.src_row[s] = a.peak_sorted[n].row;
            a.src_col[s] = a.peak_sorted[n].col;
            a.src_state[s] = kSrcLive;
            a.src_tfirst[s] = t;
            a.src_tlast[s] = t;
            a.src_tend[s] = -1;
            a.src_new[s] = 1;
            s_taken[s >> 5] |= 1u << (s & 31);  // a new source cannot be matched again
        }
        s_nnew = nnew;
        s_drop = drop;
        s_next = next;
        s_held = held;
    }
    __syncthreads();

    // ---- 5. end of monitoring, lists, events
    {
        const int per = (S + kCatThreads - 1) / kCatThreads;
        const int s0 = tid * per, s1 = min(S, s0 + per);
        int nm = 0, nn = 0, ne = 0;
        for (int s = s0; s < s1; ++s) {
            int st = a.src_state[s];
            if (st == kSrcLive) {
                ++nm;
                if (a.src_new[s]) ++nn;
                if (t - a.src_tlast[s] == a.n_mon) {
                    st = kSrcEnded;
                    a.src_state[s] = st;
                    a.src_tend[s] = t;
                }
            }
            if (st == kSrcEnded) ++ne;
            if (a.src_new[s])
                for (int r = 0; r < kRing; ++r) a.ring_t[(size_t)s * kRing + r] = INT64_MIN;
        }
        int tm, tn, te;
        int om = block_scan(nm, s_tmp, &tm);
        int on = block_scan(nn, s_tmp, &tn);
        int oe = block_scan(ne, s_tmp, &te);
        for (int s = s0; s < s1; ++s) {
            const int st = a.src_state[s];
            const bool measured = st == kSrcLive || (st == kSrcEnded && a.src_tend[s] == t);
            if (measured) a.list_measured[om++] = s;
            if (a.src_new[s]) {
                a.list_new[on] = s;
                lpf_source ev;
                ev.id = a.src_id[s];
                ev.row = a.src_row[s];
                ev.col = a.src_col[s];
                ev.event = LPF_EVENT_NEW;
                ev.t_first = a.src_tfirst[s];
                ev.t_last_det = a.src_tlast[s];
                ev.t_end = a.src_tend[s];
                a.events[on] = ev;
                ++on;
            }
            if (st == kSrcEnded) {
                a.list_ended[oe] = s;
                lpf_source ev;
                ev.id = a.src_id[s];
                ev.row = a.src_row[s];
                ev.col = a.src_col[s];
                ev.event = LPF_EVENT_ENDED;
                ev.t_first = a.src_tfirst[s];
                ev.t_last_det = a.src_tlast[s];
                ev.t_end = a.src_tend[s];
                a.events[tn + oe] = ev;
                ++oe;
            }
        }
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

hipError_t launch_catalog(lpf_ctx* c, int64_t t) {
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
    a.peak_sorted = c->buf.peak_sorted;
    a.order = c->buf.cat_order;
    a.nbr = c->buf.cat_nbr;
    a.cand = c->buf.cat_cand;
    a.kept = c->buf.cat_kept;
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
    hipLaunchKernelGGL(k_catalog, dim3(1), dim3(kCatThreads), 0, c->stream, a);
    return hipGetLastError();
}

hipError_t launch_table_init(lpf_ctx* c) {
    const int n = c->cfg.max_sources > c->d.Tc ? c->cfg.max_sources : c->d.Tc;
    hipLaunchKernelGGL(k_table_init, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->buf.src_state,
                       c->cfg.max_sources, c->buf.cache_t, c->buf.cache_rej, c->d.Tc, c->buf.status);
    return hipGetLastError();
}

}  // namespace lpf
