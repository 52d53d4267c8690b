// Batched form: many bodies, each with its own geometry, bins and forest,
// processed by one hipGraph of persistent kernels.
//
// Plan: every body is run once through the single-body calls (the bin density
// tuner times candidate densities there), which gives the exact size of every
// intermediate array; the plan reserves those sizes times 1 + margin, lays out
// per-body buffers (forest levels double-buffered, since a pass rewrites each
// level into its other buffer), and captures the whole pipeline of all bodies
// as one graph on a private stream.  Every kernel of the graph is persistent:
// a fixed grid walks the concatenated work items of all bodies (each
// workgroup first builds the per-body prefix of item counts in LDS from the
// device-side sizes, then maps items to bodies by binary search), so a run
// needs no host synchronisation.  The per-item code is the single-body code
// (kernels.hpp), so flags and link fractions are bit-identical.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "agal_internal.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace agal {
namespace batch {

using namespace kern;

constexpr int kMaxBodies = 256;
constexpr int kLv = kMaxLevels + 1;
constexpr int kScanThreads = 256;
constexpr int kScanTile = 2048;   // elements per scan tile (8 per thread)
constexpr int kMaxSeg = kMaxBodies * kLv;

// Device description of one body (pointers fixed at plan time).
struct BodyDev {
    int dim, L, Q;
    int R[3];
    float lo[3];
    float dx[kLv][3];
    float d[kMaxLevels];
    float eps[3];
    const float *verts;
    const int32_t *faces;
    int64_t Nv, F;
    float *coords, *aabb, *rec;
    int32_t *fidx;
    dev::BinGrid bins;     // off = global offsets + bin_base, ids = global ids
    int64_t nb, bin_base;
    uint32_t *keys[kLv][2];
    uint8_t *leaf[kLv][2], *mark[kLv][2], *cf[kLv][2];
    int64_t cap[kLv];
    uint8_t *pm[kLv];
    uint32_t *ftable[kLv];   // block table of level p for the face-centric flag step (null: none, or level 0)
    uint32_t *pos[kLv];
    uint32_t *mk[kLv];
    uint64_t *skey;
    float *sq;
    int32_t *sface;
    // list mode of the link step (lists != 0): parent table (null at level 0),
    // per-block node masks, candidate counts and cursors (2 x cap[L]), list
    // offsets, the lists, and each node's block
    int lists;
    int64_t per_face;
    unsigned long long *hash;
    uint32_t hmask;
    int hshift;
    unsigned long long *nmask;
    uint32_t *lwork, *loff, *lblk, *nblk;
    int32_t *list;
    uint32_t list_cap;
    uint32_t *blk_start, *blk_count, *blk_off;
    int64_t cap_nodes;
    uint64_t *key;
    float *q;
    int32_t *face;
    float *grad_q, *grad_v;
};

// Device scalars of a run.
// Staging rows of a body of node capacity cap: kRowCursors ranges (see
// ChunkRows) of this many rows each.  A range serves every kRowCursors-th
// block, so its share is about cap / kRowCursors, give or take a few standard
// deviations of a sum of block counts (each at most 64); the slack covers that.
constexpr int kRowCursors = 32;
constexpr int kCursorStride = 64;   // words: one 256-byte line per cursor
__host__ __device__ inline int64_t row_range(int64_t cap) {
    return cap / kRowCursors + cap / 20 / kRowCursors + 8 * (int64_t)sqrt((double)cap) + 128;
}

struct Ctl {
    uint32_t overflow;   // bit 0 bins, bit 1 forest level, bit 2 nodes, bit 3 candidate lists
    uint32_t err;        // bit 0 non-finite coordinate, bit 1 face index
    uint32_t balance;    // nonzero: a forest lost 2:1 balance
    uint32_t lists[2];   // medium- and big-bin list counts of the canonical order
};

// Scan segment: out[0..n] = exclusive prefix of in[0..n) (n = *n_dev or n_const).
struct Seg {
    const void *in;      // uint8 flags or uint32 counts
    uint32_t *out;
    const uint32_t *n_dev;
    int64_t n_const;
    int64_t status_base; // first status word of this segment's tiles
};

// Fill request (4-byte words).
struct Fill {
    uint32_t *p;
    int64_t words;
    uint32_t v;
};

// level m's buffer at the start of pass p (m <= p), and the one pass p writes
__device__ __forceinline__ int cur_buf(int p, int m) { return m == 0 ? 0 : ((p - m) & 1); }
__device__ __forceinline__ int new_buf(int p, int m) { return (p - m + 1) & 1; }
__device__ __forceinline__ int final_buf(int L, int m) { return m == 0 ? 0 : ((L - m) & 1); }

// Exclusive prefix of units(i), i < n (n <= kMaxSeg), into s_pre[0..n]; one wave
// computes it, the workgroup waits.  Returns the total.
template <class Units>
__device__ uint32_t lds_prefix(int n, Units units, uint32_t *s_pre) {
    if (threadIdx.x < dev::kWave) {
        uint32_t run = 0;
        for (int i0 = 0; i0 < n; i0 += dev::kWave) {
            const int i = i0 + (int)threadIdx.x;
            const uint32_t u = i < n ? units(i) : 0u;
            const uint32_t inc = dev::wave_inclusive_sum(u);
            if (i < n) s_pre[i] = run + inc - u;
            run += __shfl(inc, dev::kWave - 1, dev::kWave);
        }
        if (threadIdx.x == 0) s_pre[n] = run;
    }
    __syncthreads();
    return s_pre[n];
}

// Body of workgroup `it` in a grid laid out at plan time: pre[b] .. pre[b+1]
// are body b's workgroups (its planned capacity), so no per-launch prefix is
// needed; it is workgroup-uniform, so the search reads pre through the scalar
// cache.
__device__ __forceinline__ int body_of_wg(const uint32_t *pre, int nb, uint32_t it) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// last i with s_pre[i] <= item (the non-empty range holding item)
__device__ __forceinline__ int find_seg(const uint32_t *s_pre, int n, uint32_t item) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

#define AGAL_THREAD_ITEMS(item, total) \
    for (uint32_t item = blockIdx.x * blockDim.x + threadIdx.x; item < (total); item += gridDim.x * blockDim.x)

// ---------------------------------------------------------------------------
// set-up, fills, import, bins
// ---------------------------------------------------------------------------
__global__ void k_fill_table(const Fill *t, int n) {
    for (int e = 0; e < n; ++e) {
        uint32_t *p = t[e].p;
        const int64_t w = t[e].words;
        const uint32_t v = t[e].v;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < w; i += (int64_t)gridDim.x * blockDim.x)
            p[i] = v;
    }
}

// counts: level 0 = roots, deeper levels empty; level 0 arrays = all roots
__global__ void k_b_init(const BodyDev *bodies, int nb, uint32_t *cnt, uint32_t *cursor, Ctl *ctl) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->overflow = 0;
        ctl->err = 0;
        ctl->balance = 0;
        ctl->lists[0] = 0;
        ctl->lists[1] = 0;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < nb * kLv; i += blockDim.x) {
            const int b = i / kLv, l = i % kLv;
            cnt[i] = l == 0 ? (uint32_t)(bodies[b].R[0] * bodies[b].R[1] * bodies[b].R[2]) : 0u;
            if (l == 0)
                for (int r = 0; r < kRowCursors; ++r) cursor[((int64_t)b * kRowCursors + r) * kCursorStride] = 0;
        }
    const uint32_t total = lds_prefix(nb, [&](int b) { return (uint32_t)(bodies[b].R[0] * bodies[b].R[1] * bodies[b].R[2]); }, s_pre);
    AGAL_THREAD_ITEMS(it, total) {
        const int b = find_seg(s_pre, nb, it);
        const uint32_t i = it - s_pre[b];
        bodies[b].keys[0][0][i] = i;
        bodies[b].leaf[0][0][i] = 1;
        bodies[b].mark[0][0][i] = 0;
    }
}

template <int D>
__global__ void k_b_import(const BodyDev *bodies, int nb, Ctl *ctl) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    uint32_t bad = 0;
    const uint32_t nv = lds_prefix(nb, [&](int b) { return (uint32_t)(bodies[b].Nv * D); }, s_pre);
    AGAL_THREAD_ITEMS(it, nv) {
        const int b = find_seg(s_pre, nb, it);
        if (!isfinite(bodies[b].verts[it - s_pre[b]])) bad |= 1u;
    }
    __syncthreads();
    const uint32_t nf = lds_prefix(nb, [&](int b) { return (uint32_t)bodies[b].F; }, s_pre);
    AGAL_THREAD_ITEMS(it, nf) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &B = bodies[b];
        bad |= import_face<D>(B.verts, B.Nv, B.faces, B.F, B.coords, B.aabb, B.rec, B.fidx, it - s_pre[b]);
    }
    if (bad) atomicOr(&ctl->err, bad);
}

template <int D>
__global__ void k_b_bin_count(const BodyDev *bodies, int nb, uint32_t *count_global) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    const uint32_t nf = lds_prefix(nb, [&](int b) { return (uint32_t)bodies[b].F; }, s_pre);
    AGAL_THREAD_ITEMS(it, nf) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &B = bodies[b];
        bin_count_item<D>(B.aabb, B.F, B.bins, count_global + B.bin_base, it - s_pre[b]);
    }
}

template <int D>
__global__ void k_b_bin_scatter(const BodyDev *bodies, int nb, const uint32_t *off_global, uint32_t *cursor_global,
                                int32_t *ids, int64_t cap_ids, Ctl *ctl) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    const uint32_t nf = lds_prefix(nb, [&](int b) { return (uint32_t)bodies[b].F; }, s_pre);
    const bool over = off_global[bodies[nb - 1].bin_base + bodies[nb - 1].nb] > cap_ids;
    if (over) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctl->overflow, 1u);
        return;
    }
    AGAL_THREAD_ITEMS(it, nf) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &B = bodies[b];
        bin_scatter_item<D>(B.aabb, B.F, B.bins, off_global + B.bin_base, cursor_global + B.bin_base, ids,
                            it - s_pre[b]);
    }
}

// After an overflowing scatter, or an invalid input, every bin is made empty:
// no later kernel reads ids beyond the reserved capacity or tests a face built
// from bad input (the run reports either).
__global__ void k_b_bin_clear(uint32_t *off_global, int64_t nb_total, const Ctl *ctl) {
    if (!(ctl->overflow & 1u) && !ctl->err) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nb_total; i += (int64_t)gridDim.x * blockDim.x)
        off_global[i] = 0;
}

__global__ __launch_bounds__(64) void k_b_canon_small(int32_t *ids, const uint32_t *off_global, int64_t nb_total,
                                                      uint32_t *med_list, uint32_t *big_list, Ctl *ctl) {
    const int64_t groups = (nb_total + dev::kWave - 1) / dev::kWave;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x)
        bin_canon_group(ids, off_global, nb_total, g * dev::kWave, med_list, big_list, ctl->lists, 0u);
}

__global__ __launch_bounds__(kMedThreads) void k_b_canon_medium(int32_t *ids, const uint32_t *off_global,
                                                                const uint32_t *med_list, const Ctl *ctl) {
    const uint32_t nmed = ctl->lists[0];
    for (uint32_t i = blockIdx.x; i < nmed; i += gridDim.x) bin_canon_medium(ids, off_global, med_list[i]);
}

template <int D>
__global__ __launch_bounds__(1024) void k_b_canon_big(const BodyDev *bodies, int nb, const uint32_t *off_global,
                                                      int32_t *ids, const uint32_t *big_list, const Ctl *ctl) {
    const uint32_t nbig = ctl->lists[1];
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const int64_t gb = big_list[bi];
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (bodies[mid].bin_base <= gb) lo = mid;
            else hi = mid - 1;
        }
        const BodyDev &B = bodies[lo];
        bin_canon_big_bin<D>(B.aabb, B.F, B.bins, off_global + B.bin_base, ids, gb - B.bin_base);
    }
}

// ---------------------------------------------------------------------------
// segmented exclusive scan (decoupled look-back inside each segment)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t seg_len(const Seg &S) { return S.n_dev ? (int64_t)*S.n_dev : S.n_const; }

// Tiles per segment of one scan and their exclusive prefix, pre[0..nseg]
// (one workgroup; each thread takes consecutive segments), so that the scan's
// workgroups only look their tile up instead of each forming the prefix.
__global__ __launch_bounds__(kScanThreads) void k_b_seg_prefix(const Seg *segs, int nseg, uint32_t *pre) {
    constexpr int PER = (kMaxSeg + kScanThreads - 1) / kScanThreads;
    __shared__ uint32_t s_wsum[kScanThreads / dev::kWave];
    const int i0 = threadIdx.x * PER;
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = i0 + k;
        // every segment has at least one tile (it writes out[n] even when n = 0)
        v[k] = i < nseg ? (uint32_t)((seg_len(segs[i]) + kScanTile) / kScanTile) : 0u;
        sum += v[k];
    }
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x % dev::kWave;
    const uint32_t incl = dev::wave_inclusive_sum(sum);
    if (lane == dev::kWave - 1) s_wsum[w] = incl;
    __syncthreads();
    uint32_t run = incl - sum, tot = 0;
    for (int j = 0; j < kScanThreads / dev::kWave; ++j) {
        if (j < w) run += s_wsum[j];
        tot += s_wsum[j];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (i0 + k < nseg) pre[i0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) pre[nseg] = tot;
}

template <bool FLAGS>
__global__ __launch_bounds__(kScanThreads) void k_b_scan(const Seg *segs, int nseg, const uint32_t *pre,
                                                         uint64_t *status, uint32_t *ticket) {
    __shared__ uint32_t s_tile, s_prefix;
    __shared__ uint32_t s_wsum[kScanThreads / dev::kWave];
    const uint32_t total = pre[nseg];
    // the grid is sized for the largest scan of the plan: workgroups past this
    // scan's tiles leave before taking a ticket (tickets are one device atomic
    // on one word each, and those serialise), and the first `total` take
    // tickets 0 .. total - 1
    if (blockIdx.x >= total) return;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    if (t >= total) return;
    const int s = find_seg(pre, nseg, t);
    const Seg &S = segs[s];
    const int64_t n = seg_len(S);
    const uint32_t lt = t - pre[s];
    const int64_t base = (int64_t)lt * kScanTile + (int64_t)threadIdx.x * 8;
    uint32_t v[8];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t idx = base + i;
        uint32_t x = 0;
        if (idx < n) {
            if (FLAGS) x = static_cast<const uint8_t *>(S.in)[idx] ? 1u : 0u;
            else x = static_cast<const uint32_t *>(S.in)[idx];
        }
        v[i] = x;
        sum += x;
    }
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x % dev::kWave;
    const uint32_t incl = dev::wave_inclusive_sum(sum);
    if (lane == dev::kWave - 1) s_wsum[w] = incl;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int j = 0; j < kScanThreads / dev::kWave; ++j) {
        if (j < w) wpre += s_wsum[j];
        tot += s_wsum[j];
    }
    if (w == 0) {
        const uint32_t p = dev::lookback_wave(status + S.status_base, lt, tot);
        if (lane == 0) s_prefix = p;
    }
    __syncthreads();
    uint32_t run = s_prefix + wpre + incl - sum;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t idx = base + i;
        if (idx < n) S.out[idx] = run;
        run += v[i];
        if (idx == n - 1) S.out[n] = run;
    }
    if (n == 0 && lt == 0 && threadIdx.x == 0) S.out[0] = 0;
}

// ---------------------------------------------------------------------------
// refinement, pass p
// ---------------------------------------------------------------------------
template <int D, bool kDedup>
__global__ __launch_bounds__(64) void k_b_flag(const BodyDev *bodies, int nb, int p, const uint32_t *cnt,
                                               const uint32_t *wg_pre) {
    constexpr int BPW = D == 3 ? 1 : 4;
    {
        // one block (2D: four) per workgroup; the grid covers the planned capacity
        const uint32_t it = blockIdx.x;
        const int b = body_of_wg(wg_pre, nb, it);
        const uint32_t local = it - wg_pre[b];
        if (bodies[b].L <= p || local >= (cnt[b * kLv + p] + BPW - 1) / BPW) return;
        const BodyDev &B = bodies[b];
        FlagArgs<D> A{};
        A.faces = dev::Faces{B.coords, B.aabb, B.rec, B.F};
        A.bins = B.bins;
        A.bins.F = B.F;
        A.keys = B.keys[p][0];
        A.n = cnt[b * kLv + p];
        A.level = p;
        for (int a = 0; a < 3; ++a) {
            A.R[a] = B.R[a];
            A.lo[a] = B.lo[a];
            A.dx[a] = B.dx[p][a];
            A.eps[a] = B.eps[a];
        }
        A.h = B.d[p];
        A.cf = B.cf[p][0];
        A.pmark = B.pm[p];
        flag_wave<D, kDedup>(A, (int64_t)local * BPW);
    }
}

// Face-centric flag step of pass p (as in the single-body pass): first every
// level-p block's cell flags are zeroed and its table entry written (bodies
// with a table), then each workgroup takes 4 x 16 faces of one body.
template <int D>
__global__ void k_b_ftable(const BodyDev *bodies, int nb, int p, const uint32_t *cnt) {
    constexpr int V = (D == 3 ? 64 : 16) / 16;
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    const uint32_t total = lds_prefix(nb, [&](int b) { return bodies[b].L > p ? cnt[b * kLv + p] : 0u; }, s_pre);
    AGAL_THREAD_ITEMS(it, total) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &B = bodies[b];
        const uint32_t i = it - s_pre[b];
        uint4 *cf = reinterpret_cast<uint4 *>(B.cf[p][0]);
#pragma unroll
        for (int j = 0; j < V; ++j) cf[(int64_t)i * V + j] = make_uint4(0u, 0u, 0u, 0u);
        if (B.ftable[p]) {
            int c[3];
            dev::decode_key<D>(B.keys[p][0][i], p, B.R[0], B.R[1], c);
            B.ftable[p][((int64_t)c[2] * (B.R[1] << p) + c[1]) * (B.R[0] << p) + c[0]] = i;
        }
    }
}

template <int D, int G>
__global__ __launch_bounds__(64 * kFaceFlagWaves) void k_b_flag_faces(const BodyDev *bodies, int nb, int p,
                                                                     const uint32_t *cnt, const uint32_t *wg_pre) {
    __shared__ float s_rec[kFaceFlagWaves][G][dev::kRecFloats<D>];
    __shared__ int s_i[kFaceFlagWaves][G][kFaceFlagInts];
    const uint32_t it = blockIdx.x;
    const int b = body_of_wg(wg_pre, nb, it);
    const BodyDev &B = bodies[b];
    if (B.L <= p || cnt[b * kLv + p] == 0) return;
    const int w = (int)threadIdx.x / dev::kWave;
    FaceFlagArgs<D> A{};
    A.rec = B.rec;
    A.F = B.F;
    for (int a = 0; a < 3; ++a) {
        A.NB[a] = a < D ? B.R[a] << p : 1;
        A.lo[a] = B.lo[a];
        A.dx[a] = B.dx[p][a];
        A.eps[a] = B.eps[a];
    }
    A.table = p > 0 ? B.ftable[p] : nullptr;
    A.keys = B.keys[p][0];
    A.n = cnt[b * kLv + p];
    A.level = p;
    A.R[0] = B.R[0];
    A.R[1] = B.R[1];
    A.h = B.d[p];
    A.cf = B.cf[p][0];
    A.pmark = B.pm[p];
    flag_faces_wave<D, G>(A, ((int64_t)(it - wg_pre[b]) * kFaceFlagWaves + w) * G, s_rec[w], s_i[w]);
}

template <int D>
__global__ void k_b_ripple(const BodyDev *bodies, int nb, int p, int m, const uint32_t *cnt, Ctl *ctl) {
    constexpr int NNB = D == 3 ? 26 : 8;
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    const uint32_t total = lds_prefix(nb, [&](int b) {
        return bodies[b].L > p ? cnt[b * kLv + m] * (uint32_t)NNB : 0u; }, s_pre);
    AGAL_THREAD_ITEMS(it, total) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &B = bodies[b];
        const int cm = cur_buf(p, m), cp = cur_buf(p, m - 1);
        ripple_item<D>(B.keys[m][cm], cnt[b * kLv + m], B.pm[m], m, B.keys[m - 1][cp], cnt[b * kLv + m - 1],
                       B.leaf[m - 1][cp], B.pm[m - 1], B.R[0], B.R[1], B.R[2], &ctl->balance, it - s_pre[b]);
    }
}

// segments (body, level m <= p) for bodies still refining in pass p
__device__ __forceinline__ bool seg_live(const BodyDev *bodies, int p, int s, int &b, int &m) {
    b = s / (p + 1);
    m = s % (p + 1);
    return bodies[b].L > p;
}

__global__ void k_b_mark_parents(const BodyDev *bodies, int nb, int p, const uint32_t *cnt) {
    __shared__ uint32_t s_pre[kMaxSeg + 1];
    const int nseg = nb * (p + 1);
    const uint32_t total = lds_prefix(nseg, [&](int s) {
        int b, m;
        return seg_live(bodies, p, s, b, m) ? cnt[b * kLv + m] : 0u; }, s_pre);
    AGAL_THREAD_ITEMS(it, total) {
        const int s = find_seg(s_pre, nseg, it);
        const int b = s / (p + 1), m = s % (p + 1);
        const BodyDev &B = bodies[b];
        const int c = cur_buf(p, m);
        mark_parents_item(B.keys[m][c], B.pm[m], B.pos[m], B.leaf[m][c], B.mark[m][c], B.mk[m], it - s_pre[s]);
    }
}

template <int D>
__global__ void k_b_merge(const BodyDev *bodies, int nb, int p, const uint32_t *cnt) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    __shared__ uint32_t s_pre[kMaxSeg + 1];
    const int nseg = nb * (p + 1);
    // segment (b, m): the existing blocks of level m + 1
    const uint32_t total = lds_prefix(nseg, [&](int s) {
        int b, m;
        return seg_live(bodies, p, s, b, m) ? cnt[b * kLv + m + 1] : 0u; }, s_pre);
    AGAL_THREAD_ITEMS(it, total) {
        const int s = find_seg(s_pre, nseg, it);
        const int b = s / (p + 1), m = s % (p + 1);
        const BodyDev &B = bodies[b];
        const int c = cur_buf(p, m + 1), w = new_buf(p, m + 1);
        const uint32_t nmk = B.pos[m][cnt[b * kLv + m]];
        const bool has_cf = m + 1 <= p;
        merge_old_item<CELLS>(B.keys[m + 1][c], B.leaf[m + 1][c], B.mark[m + 1][c], has_cf ? B.cf[m + 1][c] : nullptr,
                              B.mk[m], nmk, D, B.keys[m + 1][w], B.leaf[m + 1][w], B.mark[m + 1][w],
                              has_cf ? B.cf[m + 1][w] : nullptr, it - s_pre[s], B.cap[m + 1]);
    }
    // the pass marks are consumed (the parents are marked, the scans are done):
    // clear them for the next pass, which finds them zero as the first pass
    // finds them from the plan's initial clearing
    __syncthreads();
    const uint32_t words = lds_prefix(nseg, [&](int s) {
        int b, m;
        return seg_live(bodies, p, s, b, m) ? (uint32_t)((bodies[b].cap[m] + 3) / 4) : 0u; }, s_pre);
    AGAL_THREAD_ITEMS(it, words) {
        const int s = find_seg(s_pre, nseg, it);
        const int b = s / (p + 1), m = s % (p + 1);
        reinterpret_cast<uint32_t *>(bodies[b].pm[m])[it - s_pre[s]] = 0u;
    }
}

template <int D>
__global__ void k_b_children(const BodyDev *bodies, int nb, int p, const uint32_t *cnt) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    __shared__ uint32_t s_pre[kMaxSeg + 1];
    const int nseg = nb * (p + 1);
    const uint32_t total = lds_prefix(nseg, [&](int s) {
        int b, m;
        return seg_live(bodies, p, s, b, m) ? (bodies[b].pos[m][cnt[b * kLv + m]] << D) : 0u; }, s_pre);
    AGAL_THREAD_ITEMS(it, total) {
        const int s = find_seg(s_pre, nseg, it);
        const int b = s / (p + 1), m = s % (p + 1);
        const BodyDev &B = bodies[b];
        const int c = cur_buf(p, m + 1), w = new_buf(p, m + 1);
        const bool has_cf = m + 1 <= p;
        children_item<CELLS>(B.mk[m], B.keys[m + 1][c], cnt[b * kLv + m + 1], D, B.keys[m + 1][w],
                             B.leaf[m + 1][w], B.mark[m + 1][w], has_cf ? B.cf[m + 1][w] : nullptr, it - s_pre[s],
                             B.cap[m + 1]);
    }
}

// new level sizes after pass p (clamped to capacity)
template <int D>
__global__ void k_b_counts(const BodyDev *bodies, int nb, int p, uint32_t *cnt, Ctl *ctl) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nb; s += gridDim.x * blockDim.x) {
        const BodyDev &B = bodies[s];
        if (B.L <= p) continue;
        uint32_t add[kLv];
        for (int m = 0; m <= p; ++m) add[m] = B.pos[m][cnt[s * kLv + m]] << D;
        for (int m = 0; m <= p; ++m) {
            int64_t nn = (int64_t)cnt[s * kLv + m + 1] + add[m];
            if (nn > B.cap[m + 1]) {
                atomicOr(&ctl->overflow, 2u);
                nn = B.cap[m + 1];
            }
            cnt[s * kLv + m + 1] = (uint32_t)nn;
        }
    }
}

// ---------------------------------------------------------------------------
// link fractions, compaction, adjoint
// ---------------------------------------------------------------------------
// Staging rows handed out in block-sized chunks.  A body's staging area is
// kRowCursors ranges of row_range(cap) rows, each with its own cursor in its
// own 256-byte line, and block blk draws from range blk mod kRowCursors.
// (One counter per body took every block's atomic at one address; those
// serialise: 86 us of a 206 us pass over a 20,480-face sphere.)
struct ChunkRows {
    uint32_t *blk_start, *blk_count, *cursor;   // cursor: this body's kRowCursors counters
    int64_t cap;                                // node capacity of the body
    Ctl *ctl;
    __device__ int64_t rows(int64_t blk, uint32_t c) {
        const int r = (int)(blk % kRowCursors);
        const int64_t range = row_range(cap);
        const uint32_t start = c ? atomicAdd(&cursor[r * kCursorStride], c) : 0u;
        if ((int64_t)start + c > range) {
            atomicOr(&ctl->overflow, 4u);
            blk_count[blk] = 0;
            blk_start[blk] = 0;
            return -1;
        }
        const int64_t row = r * range + start;
        blk_start[blk] = (uint32_t)row;
        blk_count[blk] = c;
        return row;
    }
};

template <int D, int Q>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_b_links(const BodyDev *bodies, int nb, const uint32_t *cnt,
                                                uint32_t *cursor, Ctl *ctl, const uint32_t *wg_pre) {
    constexpr int BPW = D == 3 ? 1 : 4;
    {
        const uint32_t it = blockIdx.x;
        const int b = body_of_wg(wg_pre, nb, it);
        const BodyDev &B = bodies[b];
        const int L = B.L;
        const uint32_t local = it - wg_pre[b];
        if (B.Q != Q || B.lists || local >= (cnt[b * kLv + L] + BPW - 1) / BPW) return;
        LinkArgs<D, Q> A{};
        A.faces = dev::Faces{B.coords, B.aabb, B.rec, B.F};
        A.bins = B.bins;
        A.bins.F = B.F;
        A.keys = B.keys[L][final_buf(L, L)];
        A.n = cnt[b * kLv + L];
        A.level = L;
        for (int a = 0; a < 3; ++a) {
            A.R[a] = B.R[a];
            A.lo[a] = B.lo[a];
            A.dx[a] = B.dx[L][a];
            A.eps[a] = B.eps[a];
        }
        A.node_key = B.skey;
        A.q = B.sq;
        A.face = B.sface;
        ChunkRows out{B.blk_start, B.blk_count, cursor + (int64_t)b * kRowCursors * kCursorStride, B.cap_nodes, ctl};
        links_wave<D, Q>(A, (int64_t)local * BPW, out);
    }
}

// Nodes of each body; more than its capacity is reported and clamped (the
// compaction then leaves out the blocks that would not fit).
__global__ void k_b_nodes(const BodyDev *bodies, int nb, const uint32_t *cnt, uint32_t *nodes, Ctl *ctl) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
        const uint32_t n = bodies[b].blk_off[cnt[b * kLv + bodies[b].L]];
        const bool over = (int64_t)n > bodies[b].cap_nodes;
        if (over) atomicOr(&ctl->overflow, 4u);
        // list mode writes rows by node index: a body over capacity gets none
        nodes[b] = bodies[b].lists ? (over ? 0u : n) : (uint32_t)std::min<int64_t>(n, bodies[b].cap_nodes);
    }
}

template <int D, int Q>
__global__ __launch_bounds__(64) void k_b_compact(const BodyDev *bodies, int nb, const uint32_t *cnt) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    const uint32_t total = lds_prefix(nb, [&](int b) {
        return bodies[b].Q == Q && !bodies[b].lists ? cnt[b * kLv + bodies[b].L] : 0u; }, s_pre);
    for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &B = bodies[b];
        const uint32_t i = it - s_pre[b];
        const uint32_t c = B.blk_count[i], dst = B.blk_off[i];
        if ((int64_t)dst + c > B.cap_nodes) continue;   // over capacity (reported by k_b_nodes)
        compact_block<Q>((int)c, B.blk_start[i], dst, B.skey, B.sq, B.sface, B.key, B.q, B.face);
    }
}

// ---- list mode ------------------------------------------------------------
// The single-body list build and passes (kernels.hpp), body by body: blocks
// and faces are mapped to bodies through per-body prefixes, the wave-per-unit
// kernels through workgroup offsets laid out at plan time.
template <int D>
__device__ __forceinline__ BlockFind body_find(const BodyDev &X, uint32_t n) {
    BlockFind B{};
    B.hash = X.hash;
    B.hmask = X.hmask;
    B.hshift = X.hshift;
    B.level = X.L;
    for (int a = 0; a < 3; ++a) B.R[a] = X.R[a];
    B.keys = X.keys[X.L][final_buf(X.L, X.L)];
    B.n = n;
    return B;
}

template <int D, int Q>
__device__ __forceinline__ LinkArgs<D, Q> body_link_args(const BodyDev &X, uint32_t n) {
    LinkArgs<D, Q> A{};
    A.faces = dev::Faces{X.coords, X.aabb, X.rec, X.F};
    A.bins = X.bins;
    A.bins.F = X.F;
    A.keys = X.keys[X.L][final_buf(X.L, X.L)];
    A.n = n;
    A.level = X.L;
    for (int a = 0; a < 3; ++a) {
        A.R[a] = X.R[a];
        A.lo[a] = X.lo[a];
        A.dx[a] = X.dx[X.L][a];
        A.eps[a] = X.eps[a];
    }
    A.loff = X.loff;
    A.list = X.list;
    A.list_cap = X.list_cap;
    A.node_key = X.key;
    A.q = X.q;
    A.face = X.face;
    return A;
}

template <int D>
__global__ void k_b_link_blocks(const BodyDev *bodies, int nb, const uint32_t *cnt) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    const uint32_t total = lds_prefix(nb, [&](int b) {
        return bodies[b].lists ? cnt[b * kLv + bodies[b].L] : 0u; }, s_pre);
    AGAL_THREAD_ITEMS(it, total) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &X = bodies[b];
        link_block_item<D>(X.keys[X.L][final_buf(X.L, X.L)], it - s_pre[b], X.hash, X.hmask, X.hshift, X.nmask);
    }
}

template <int D, bool kScatter>
__global__ __launch_bounds__(64) void k_b_link_faces(const BodyDev *bodies, int nb, const uint32_t *cnt, Ctl *ctl,
                                                     const uint32_t *wg_pre) {
    const uint32_t it = blockIdx.x;
    const int b = body_of_wg(wg_pre, nb, it);
    const BodyDev &X = bodies[b];
    if (!X.lists) return;
    const uint32_t n = cnt[b * kLv + X.L];
    LinkFaceGrid G{};
    for (int a = 0; a < 3; ++a) {
        G.lo[a] = X.lo[a];
        G.dx[a] = X.dx[X.L][a];
        G.m[a] = 2.0 * (double)X.eps[a];
        G.NB[a] = a < D ? (X.R[a] << X.L) : 1;
    }
    const BlockFind B = body_find<D>(X, n);
    const int64_t f0 = (int64_t)(it - wg_pre[b]) * kLinkFaceG;
    link_faces_wave<D, kScatter>(X.aabb, X.F, G, B, X.per_face, X.lwork, X.loff, X.lwork + X.cap[X.L], X.list,
                                 X.lblk, X.list_cap, f0, kScatter ? nullptr : &ctl->overflow);
}

template <int D, int Q>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_b_links_nodes(const BodyDev *bodies, int nb, const uint32_t *cnt,
                                                      const uint32_t *wg_pre) {
    const uint32_t it = blockIdx.x;
    const int b = body_of_wg(wg_pre, nb, it);
    const BodyDev &X = bodies[b];
    if (X.Q != Q || !X.lists) return;
    const LinkArgs<D, Q> A = body_link_args<D, Q>(X, cnt[b * kLv + X.L]);
    links_nodes_entries<D, Q>(A, X.lblk, X.nmask, it - wg_pre[b], wg_pre[b + 1] - wg_pre[b]);
}

// Node counts per block (the links scan lays out the rows), and the list
// length checked against its capacity.
__global__ void k_b_popc(const BodyDev *bodies, int nb, const uint32_t *cnt, Ctl *ctl) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    const uint32_t total = lds_prefix(nb, [&](int b) {
        return bodies[b].lists ? cnt[b * kLv + bodies[b].L] : 0u; }, s_pre);
    AGAL_THREAD_ITEMS(it, total) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &X = bodies[b];
        const uint32_t i = it - s_pre[b];
        X.blk_count[i] = (uint32_t)__popcll(X.nmask[i]);
        if (i == 0 && X.loff[cnt[b * kLv + X.L]] > X.list_cap) atomicOr(&ctl->overflow, 8u);
    }
}

template <int D>
__global__ void k_b_node_map(const BodyDev *bodies, int nb, const uint32_t *cnt, const uint32_t *nodes) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    // items: chunks of 64 blocks of one body, one per wave at a time
    const uint32_t total = lds_prefix(nb, [&](int b) {
        return bodies[b].lists && nodes[b] ? (cnt[b * kLv + bodies[b].L] + 63u) / 64u : 0u; }, s_pre);
    const uint32_t w0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) / 64u));
    for (uint32_t it = w0; it < total; it += gridDim.x * (blockDim.x / 64u)) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &X = bodies[b];
        node_map_chunk<D>(X.nmask, X.blk_off, X.keys[X.L][final_buf(X.L, X.L)], (int64_t)(it - s_pre[b]) * 64,
                          cnt[b * kLv + X.L], X.nblk, X.key);
    }
}

template <int D, int Q>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_b_links_rows(
    const BodyDev *bodies, int nb, const uint32_t *cnt, const uint32_t *nodes, const uint32_t *wg_pre) {
    const uint32_t it = blockIdx.x;
    const int b = body_of_wg(wg_pre, nb, it);
    const BodyDev &X = bodies[b];
    const uint32_t local = it - wg_pre[b];
    if (X.Q != Q || !X.lists || (int64_t)local * kRowNodes >= (int64_t)nodes[b]) return;
    const LinkArgs<D, Q> A = body_link_args<D, Q>(X, cnt[b * kLv + X.L]);
    links_rows_nodes<D, Q>(A, X.lblk, X.nblk, X.key, nodes[b], local);
}

template <int D, int Q>
__global__ __launch_bounds__(kAdjThreads) void k_b_adjoint(const BodyDev *bodies, int nb, const uint32_t *nodes) {
    __shared__ uint32_t s_pre[kMaxBodies + 1];
    const uint32_t total = lds_prefix(nb, [&](int b) {
        return bodies[b].Q == Q ? (nodes[b] + kAdjThreads - 1) / kAdjThreads : 0u; }, s_pre);
    for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int b = find_seg(s_pre, nb, it);
        const BodyDev &B = bodies[b];
        AdjArgs<D, Q> A{};
        A.rec = B.rec;
        A.F = B.F;
        A.fidx = B.fidx;
        A.node_key = B.key;
        A.face = B.face;
        A.gq = B.grad_q;
        A.n = nodes[b];
        A.level = B.L;
        for (int a = 0; a < 3; ++a) {
            A.R[a] = B.R[a];
            A.lo[a] = B.lo[a];
            A.dx[a] = B.dx[B.L][a];
        }
        A.grad = B.grad_v;
        adjoint_tile<D, Q>(A, (int64_t)(it - s_pre[b]) * kAdjThreads);
    }
}

}  // namespace batch
}  // namespace agal

// ===========================================================================
// host side
// ===========================================================================
namespace agal {
namespace batch {

struct BodyHost {
    agal_body_desc desc;
    std::vector<float> d_spec;
    int B = 0;
    int64_t nb = 0;
    int64_t P = 0;
    int64_t n[kLv] = {};
    int64_t nodes = 0;
    double tune_ms = 0;
    float max_extent[3] = {};   // largest face box extent per axis (from the sizing run)
    bool lists = false;         // the single-body link step takes list mode
    int64_t list_entries = 0;   // candidate-list entries of the sizing run
};

}  // namespace batch
}  // namespace agal

struct agal_batch_t {
    agal_context ctx = nullptr;
    hipStream_t cap_stream = nullptr;
    int nb = 0, dim = 3, Lmax = 0;
    std::vector<agal::batch::BodyHost> host;
    std::vector<agal::batch::BodyDev> bodies;
    agal::batch::BodyDev *d_bodies = nullptr;
    std::vector<void *> owned;
    uint32_t *d_cnt = nullptr, *d_nodes = nullptr, *d_cursor = nullptr;
    agal::batch::Ctl *d_ctl = nullptr;
    uint32_t *d_bin_count = nullptr, *d_bin_off = nullptr, *d_bin_cursor = nullptr, *d_big = nullptr, *d_med = nullptr;
    int32_t *d_ids = nullptr;
    int64_t nb_total = 0, cap_ids = 0;
    uint64_t *d_status = nullptr;
    int64_t status_words = 0;
    std::vector<agal::batch::Seg> seg_store;
    agal::batch::Seg *d_segs = nullptr;
    agal::batch::Fill *d_fills = nullptr;
    int n_fill_init = 0;
    std::vector<int> pass_seg_off, pass_seg_n;
    uint32_t *d_tickets = nullptr;   // one look-back ticket per scan of a run
    uint32_t *d_segpre = nullptr;    // per scan: tile prefix over its segments (kMaxSeg + 1 words)
    int links_seg_off = 0, bins_seg_off = 0, lists_seg_off = 0;
    int fill_pass_base = 0;
    int wg_per_cu = 4, n_cu = 256;
    bool with_adjoint = false;
    unsigned flag_grid[agal::kMaxLevels] = {};   // workgroups of the flag kernel per pass (from capacities)
    bool flag_dedup[agal::kMaxLevels] = {};      // the flag pass takes the deduplicating walker
    bool flag_faces[agal::kMaxLevels] = {};      // the flag pass is face-centric (every body's table fits)
    unsigned fflag_grid = 0;                     // workgroups of the face-centric flag kernel (4 G faces each)
    int fflag_g = 16;                            // faces per wave of that kernel (face_flag_g of all faces)
    unsigned links_grid[28] = {};                // workgroups of the walk-mode q kernel per lattice
    bool any_lists = false;                      // some body takes list mode
    unsigned lfaces_grid = 0;                    // waves of the list build (kLinkFaceG faces each)
    unsigned nodes_grid[28] = {};                // waves of the node pass per lattice
    unsigned rows_grid[28] = {};                 // waves of the row pass per lattice
    uint32_t *d_wg_pre = nullptr;   // per flag pass, per lattice (9, 19, 27), then per face group: nb + 1 offsets
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint32_t> h_cnt, h_nodes;
    uint32_t h_overflow = 0, h_err = 0;
    bool have_status = false;
};

namespace agal {
namespace batch {

template <class T>
static agal_status own(agal_batch bt, T **p, size_t count) {
    count = ((count * sizeof(T) + 15) / 16) * 16 / sizeof(T) + 1;   // padded: fills work in 4-byte words
    AGAL_TRY(dev_alloc(bt->ctx->mem, p, count, bt->cap_stream));
    bt->owned.push_back(*p);
    return AGAL_OK;
}

static int64_t margin(int64_t n, float m) { return (int64_t)std::ceil((double)n * (1.0 + m)) + 64; }

// --- tuner cache: one "dim logF roots levels lattice B" line per entry ----
static std::string bucket_key(const agal_body_desc &d) {
    const int lf = (int)std::floor(std::log2((double)std::max<int64_t>(1, d.n_faces)));
    char buf[128];
    snprintf(buf, sizeof buf, "%d %d %d %d %d %d", d.dim, lf, d.forest.roots[0], d.forest.roots[1],
             d.dim == 3 ? d.forest.roots[2] : 1, d.forest.n_levels);
    return std::string(buf) + " " + std::to_string(d.lattice);
}

static void cache_load(const char *path, std::map<std::string, int> &m) {
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        int a[7], B;
        if (sscanf(line, "%d %d %d %d %d %d %d %d", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5], &a[6], &B) == 8) {
            char k[128];
            snprintf(k, sizeof k, "%d %d %d %d %d %d %d", a[0], a[1], a[2], a[3], a[4], a[5], a[6]);
            m[k] = B;
        }
    }
    fclose(f);
}

static void cache_store(const char *path, const std::map<std::string, int> &m) {
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "# dim log2(faces) roots_x roots_y roots_z levels lattice -> bins per axis\n");
    for (auto &kv : m) fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
    fclose(f);
}

// Starting density: about a dozen faces per occupied bin for a closed surface
// of area ~0.5 in the unit cube (2D: curve of length ~1.6).
static int default_bins(const agal_body_desc &d) {
    const double F = (double)d.n_faces;
    double B = d.dim == 3 ? std::sqrt(F / 6.0) : F / 8.0;
    int b = 1;
    while (b < B) b <<= 1;
    return std::max(4, std::min(b, 512));
}

// One single-body pass (import, bins, refine, links); returns sizes and the
// time of the bins + refine + links calls measured with events.
static agal_status size_body(agal_context ctx, const agal_body_desc &d, int B, hipStream_t s, BodyHost &h,
                             double *ms) {
    agal_geom g = nullptr;
    agal_bins bn = nullptr;
    agal_forest fo = nullptr;
    agal_links lk = nullptr;
    agal_status st = agal_import_faces(ctx, d.dim, d.d_vertices, d.n_vertices, d.d_faces, d.n_faces, s, &g);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == AGAL_OK && ms) {
        AGAL_TRY_HIP(hipEventCreate(&e0));
        AGAL_TRY_HIP(hipEventCreate(&e1));
        AGAL_TRY_HIP(hipEventRecord(e0, s));
    }
    if (st == AGAL_OK) st = agal_bin_faces(g, d.forest.lo, d.forest.hi, B, s, &bn);
    if (st == AGAL_OK) st = agal_near_wall_refine(g, bn, &d.forest, s, &fo);
    if (st == AGAL_OK) st = agal_link_fractions(g, bn, fo, d.lattice, s, &lk);
    if (st == AGAL_OK && ms) {
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float t = 0;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st == AGAL_OK) {
        h.B = B;
        h.nb = bn->nb;
        h.P = bn->P;
        for (int l = 0; l <= fo->L; ++l) h.n[l] = fo->lev[l].n;
        h.nodes = lk->n;
        for (int a = 0; a < 3; ++a) h.max_extent[a] = g->max_extent[a];
        LinkListPlan lp;
        st = link_list_plan(g, fo, s, &lp);
        h.lists = lp.lists;
        h.list_entries = lp.entries;
    }
    agal_destroy_links(lk);
    agal_destroy_forest(fo);
    agal_destroy_bins(bn);
    agal_destroy_geom(g);
    return st;
}

template <int D>
static agal_status capture(agal_batch bt) {
    hipStream_t s = bt->cap_stream;
    const int nb = bt->nb;
    const unsigned G = (unsigned)(bt->wg_per_cu * bt->n_cu);
    const unsigned G64 = G * 4;   // single-wave workgroups: four per CU slot of a 256-thread one
    BodyDev *B = bt->d_bodies;
    AGAL_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_fill_table, dim3(G), dim3(256), 0, s, bt->d_fills, bt->n_fill_init);
    hipLaunchKernelGGL(k_b_init, dim3(G), dim3(256), 0, s, B, nb, bt->d_cnt, bt->d_cursor, bt->d_ctl);
    hipLaunchKernelGGL(k_b_import<D>, dim3(G), dim3(256), 0, s, B, nb, bt->d_ctl);
    hipLaunchKernelGGL(k_b_bin_count<D>, dim3(G), dim3(256), 0, s, B, nb, bt->d_bin_count);
    // scans use ticket order; each scan resets the ticket afterwards via the next fill
    // every scan starts from cleared status words and ticket (two fill entries);
    // its grid is the largest tile count any scan of the plan can need
    // scan i has its own status words and ticket, all cleared by the first fill
    auto scan = [&](int idx, int seg_off, int nseg, bool flags) {
        const unsigned grid = (unsigned)bt->status_words;
        uint64_t *st = bt->d_status + (size_t)idx * bt->status_words;
        uint32_t *tk = bt->d_tickets + idx;
        uint32_t *pre = bt->d_segpre + (size_t)idx * (kMaxSeg + 1);
        hipLaunchKernelGGL(k_b_seg_prefix, dim3(1), dim3(kScanThreads), 0, s, bt->d_segs + seg_off, nseg, pre);
        if (flags)
            hipLaunchKernelGGL(k_b_scan<true>, dim3(grid), dim3(kScanThreads), 0, s, bt->d_segs + seg_off, nseg, pre,
                               st, tk);
        else
            hipLaunchKernelGGL(k_b_scan<false>, dim3(grid), dim3(kScanThreads), 0, s, bt->d_segs + seg_off, nseg, pre,
                               st, tk);
    };
    scan(0, bt->bins_seg_off, 1, false);
    hipLaunchKernelGGL(k_b_bin_scatter<D>, dim3(G), dim3(256), 0, s, B, nb, bt->d_bin_off, bt->d_bin_cursor, bt->d_ids,
                       bt->cap_ids, bt->d_ctl);
    hipLaunchKernelGGL(k_b_bin_clear, dim3(G), dim3(256), 0, s, bt->d_bin_off, bt->nb_total, bt->d_ctl);
    hipLaunchKernelGGL(k_b_canon_small, dim3(G64), dim3(64), 0, s, bt->d_ids, bt->d_bin_off, bt->nb_total, bt->d_med,
                       bt->d_big, bt->d_ctl);
    hipLaunchKernelGGL(k_b_canon_medium, dim3(G), dim3(kMedThreads), 0, s, bt->d_ids, bt->d_bin_off, bt->d_med,
                       bt->d_ctl);
    hipLaunchKernelGGL(k_b_canon_big<D>, dim3(std::min<unsigned>(G, 256)), dim3(1024), 0, s, B, nb, bt->d_bin_off,
                       bt->d_ids, bt->d_big, bt->d_ctl);
    for (int p = 0; p < bt->Lmax; ++p) {
        if (bt->flag_faces[p]) {
            hipLaunchKernelGGL(k_b_ftable<D>, dim3(G), dim3(256), 0, s, B, nb, p, bt->d_cnt);
            const uint32_t *pre = bt->d_wg_pre + (size_t)(kLv + 3) * (nb + 1);
            if (bt->fflag_g == 16)
                hipLaunchKernelGGL((k_b_flag_faces<D, 16>), dim3(bt->fflag_grid), dim3(64 * kFaceFlagWaves), 0, s, B,
                                   nb, p, bt->d_cnt, pre);
            else if (bt->fflag_g == 8)
                hipLaunchKernelGGL((k_b_flag_faces<D, 8>), dim3(bt->fflag_grid), dim3(64 * kFaceFlagWaves), 0, s, B,
                                   nb, p, bt->d_cnt, pre);
            else
                hipLaunchKernelGGL((k_b_flag_faces<D, 4>), dim3(bt->fflag_grid), dim3(64 * kFaceFlagWaves), 0, s, B,
                                   nb, p, bt->d_cnt, pre);
        } else if (bt->flag_dedup[p])
            hipLaunchKernelGGL((k_b_flag<D, true>), dim3(bt->flag_grid[p]), dim3(64), 0, s, B, nb, p, bt->d_cnt,
                               bt->d_wg_pre + (size_t)p * (nb + 1));
        else
            hipLaunchKernelGGL((k_b_flag<D, false>), dim3(bt->flag_grid[p]), dim3(64), 0, s, B, nb, p, bt->d_cnt,
                               bt->d_wg_pre + (size_t)p * (nb + 1));
        for (int m = p; m >= 1; --m)
            hipLaunchKernelGGL(k_b_ripple<D>, dim3(G), dim3(256), 0, s, B, nb, p, m, bt->d_cnt, bt->d_ctl);
        scan(1 + p, bt->pass_seg_off[p], bt->pass_seg_n[p], true);
        hipLaunchKernelGGL(k_b_mark_parents, dim3(G), dim3(256), 0, s, B, nb, p, bt->d_cnt);
        hipLaunchKernelGGL(k_b_merge<D>, dim3(G), dim3(256), 0, s, B, nb, p, bt->d_cnt);
        hipLaunchKernelGGL(k_b_children<D>, dim3(G), dim3(256), 0, s, B, nb, p, bt->d_cnt);
        hipLaunchKernelGGL(k_b_counts<D>, dim3(1), dim3(256), 0, s, B, nb, p, bt->d_cnt, bt->d_ctl);
    }
    if (bt->any_lists) {
        const uint32_t *fpre = bt->d_wg_pre + (size_t)(kLv + 4) * (nb + 1);
        hipLaunchKernelGGL(k_b_link_blocks<D>, dim3(G), dim3(256), 0, s, B, nb, bt->d_cnt);
        hipLaunchKernelGGL((k_b_link_faces<D, false>), dim3(bt->lfaces_grid), dim3(64), 0, s, B, nb, bt->d_cnt,
                           bt->d_ctl, fpre);
        scan(2 + bt->Lmax, bt->lists_seg_off, nb, false);
        hipLaunchKernelGGL((k_b_link_faces<D, true>), dim3(bt->lfaces_grid), dim3(64), 0, s, B, nb, bt->d_cnt,
                           bt->d_ctl, fpre);
        if (D == 3) {
            if (bt->nodes_grid[19])
                hipLaunchKernelGGL((k_b_links_nodes<3, 19>), dim3(bt->nodes_grid[19]), dim3(64), 0, s, B, nb,
                                   bt->d_cnt, bt->d_wg_pre + (size_t)(kLv + 6) * (nb + 1));
            if (bt->nodes_grid[27])
                hipLaunchKernelGGL((k_b_links_nodes<3, 27>), dim3(bt->nodes_grid[27]), dim3(64), 0, s, B, nb,
                                   bt->d_cnt, bt->d_wg_pre + (size_t)(kLv + 7) * (nb + 1));
        } else if (bt->nodes_grid[9]) {
            hipLaunchKernelGGL((k_b_links_nodes<2, 9>), dim3(bt->nodes_grid[9]), dim3(64), 0, s, B, nb, bt->d_cnt,
                               bt->d_wg_pre + (size_t)(kLv + 5) * (nb + 1));
        }
        hipLaunchKernelGGL(k_b_popc, dim3(G), dim3(256), 0, s, B, nb, bt->d_cnt, bt->d_ctl);
    }
    if (D == 3) {
        if (bt->links_grid[19])
            hipLaunchKernelGGL((k_b_links<3, 19>), dim3(bt->links_grid[19]), dim3(64), 0, s, B, nb, bt->d_cnt,
                               bt->d_cursor, bt->d_ctl, bt->d_wg_pre + (size_t)(kLv + 1) * (nb + 1));
        if (bt->links_grid[27])
            hipLaunchKernelGGL((k_b_links<3, 27>), dim3(bt->links_grid[27]), dim3(64), 0, s, B, nb, bt->d_cnt,
                               bt->d_cursor, bt->d_ctl, bt->d_wg_pre + (size_t)(kLv + 2) * (nb + 1));
    } else {
        if (bt->links_grid[9])
            hipLaunchKernelGGL((k_b_links<2, 9>), dim3(bt->links_grid[9]), dim3(64), 0, s, B, nb, bt->d_cnt,
                               bt->d_cursor, bt->d_ctl, bt->d_wg_pre + (size_t)(kLv + 0) * (nb + 1));
    }
    scan(1 + bt->Lmax, bt->links_seg_off, nb, false);
    hipLaunchKernelGGL(k_b_nodes, dim3(1), dim3(256), 0, s, B, nb, bt->d_cnt, bt->d_nodes, bt->d_ctl);
    if (bt->any_lists) {
        hipLaunchKernelGGL(k_b_node_map<D>, dim3(G), dim3(256), 0, s, B, nb, bt->d_cnt, bt->d_nodes);
        if (D == 3) {
            if (bt->rows_grid[19])
                hipLaunchKernelGGL((k_b_links_rows<3, 19>), dim3(bt->rows_grid[19]), dim3(64), 0, s, B, nb,
                                   bt->d_cnt, bt->d_nodes, bt->d_wg_pre + (size_t)(kLv + 9) * (nb + 1));
            if (bt->rows_grid[27])
                hipLaunchKernelGGL((k_b_links_rows<3, 27>), dim3(bt->rows_grid[27]), dim3(64), 0, s, B, nb,
                                   bt->d_cnt, bt->d_nodes, bt->d_wg_pre + (size_t)(kLv + 10) * (nb + 1));
        } else if (bt->rows_grid[9]) {
            hipLaunchKernelGGL((k_b_links_rows<2, 9>), dim3(bt->rows_grid[9]), dim3(64), 0, s, B, nb, bt->d_cnt,
                               bt->d_nodes, bt->d_wg_pre + (size_t)(kLv + 8) * (nb + 1));
        }
    }
    if (D == 3) {
        hipLaunchKernelGGL((k_b_compact<3, 19>), dim3(G64), dim3(64), 0, s, B, nb, bt->d_cnt);
        hipLaunchKernelGGL((k_b_compact<3, 27>), dim3(G64), dim3(64), 0, s, B, nb, bt->d_cnt);
    } else {
        hipLaunchKernelGGL((k_b_compact<2, 9>), dim3(G64), dim3(64), 0, s, B, nb, bt->d_cnt);
    }
    if (bt->with_adjoint) {
        if (D == 3) {
            hipLaunchKernelGGL((k_b_adjoint<3, 19>), dim3(G), dim3(kAdjThreads), 0, s, B, nb, bt->d_nodes);
            hipLaunchKernelGGL((k_b_adjoint<3, 27>), dim3(G), dim3(kAdjThreads), 0, s, B, nb, bt->d_nodes);
        } else {
            hipLaunchKernelGGL((k_b_adjoint<2, 9>), dim3(G), dim3(kAdjThreads), 0, s, B, nb, bt->d_nodes);
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(AGAL_EHIP, "batch capture failed: %s / %s", hipGetErrorString(e1), hipGetErrorString(e2));
    }
    hipGraphExec_t exec = nullptr;
    hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(AGAL_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
    }
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->graph = graph;
    bt->exec = exec;
    return AGAL_OK;
}

static agal_status time_graph(agal_batch bt, int reps, double *ms) {
    hipEvent_t e0, e1;
    AGAL_TRY_HIP(hipEventCreate(&e0));
    AGAL_TRY_HIP(hipEventCreate(&e1));
    AGAL_TRY_HIP(hipGraphLaunch(bt->exec, bt->cap_stream));
    AGAL_TRY_HIP(hipEventRecord(e0, bt->cap_stream));
    for (int r = 0; r < reps; ++r) AGAL_TRY_HIP(hipGraphLaunch(bt->exec, bt->cap_stream));
    AGAL_TRY_HIP(hipEventRecord(e1, bt->cap_stream));
    AGAL_TRY_HIP(hipEventSynchronize(e1));
    float t = 0;
    AGAL_TRY_HIP(hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return AGAL_OK;
}

template <int D>
static agal_status plan(agal_batch bt, const agal_tune_opts &opt, hipStream_t user) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    agal_context ctx = bt->ctx;
    const float mg = opt.capacity_margin > 0 ? opt.capacity_margin : 0.25f;
    // ---- size every body (and tune its bin density) --------------------------
    std::map<std::string, int> cache;
    cache_load(opt.cache_path, cache);
    bool cache_dirty = false;
    for (int b = 0; b < bt->nb; ++b) {
        BodyHost &h = bt->host[b];
        const agal_body_desc &d = h.desc;
        int B = d.bins;
        if (B <= 0) {
            const std::string k = bucket_key(d);
            auto it = cache.find(k);
            if (it != cache.end()) {
                B = it->second;
            } else if (opt.tune_bins) {
                const int B0 = default_bins(d);
                double best = 1e30;
                int bestB = B0;
                for (int cand : {B0 / 2, B0, B0 * 2}) {
                    if (cand < 2 || (int64_t)cand * cand * (D == 3 ? cand : 1) > ((int64_t)1 << 27)) continue;
                    double t1 = 0, t2 = 0;
                    BodyHost tmp;
                    AGAL_TRY(size_body(ctx, d, cand, user, tmp, &t1));
                    AGAL_TRY(size_body(ctx, d, cand, user, tmp, &t2));
                    const double t = std::min(t1, t2);
                    if (t < best) {
                        best = t;
                        bestB = cand;
                    }
                }
                B = bestB;
                h.tune_ms = best;
                cache[k] = B;
                cache_dirty = true;
            } else {
                B = default_bins(d);
            }
        }
        AGAL_TRY(size_body(ctx, d, B, user, h, nullptr));
    }
    if (cache_dirty) cache_store(opt.cache_path, cache);
    AGAL_TRY_HIP(hipStreamSynchronize(user));

    // ---- buffers -------------------------------------------------------------
    bt->bodies.assign(bt->nb, BodyDev{});
    bt->Lmax = 0;
    int64_t bin_base = 0, cap_ids = 0;
    for (int b = 0; b < bt->nb; ++b) {
        BodyHost &h = bt->host[b];
        const agal_body_desc &d = h.desc;
        BodyDev &X = bt->bodies[b];
        X.dim = D;
        X.L = d.forest.n_levels;
        X.Q = d.lattice;
        bt->Lmax = std::max(bt->Lmax, X.L);
        for (int a = 0; a < 3; ++a) {
            X.R[a] = a < D ? d.forest.roots[a] : 1;
            X.lo[a] = a < D ? d.forest.lo[a] : 0.0f;
            const float hi = a < D ? d.forest.hi[a] : 1.0f;
            for (int l = 0; l <= X.L; ++l) X.dx[l][a] = (hi - X.lo[a]) / (float)(4 * X.R[a] * (1 << l));
            const float sc = std::max(1.0f, std::max(std::fabs(X.lo[a]), std::fabs(hi)));
            X.eps[a] = dev::kEps * sc;
            X.bins.lo[a] = a < D ? d.forest.lo[a] : 0.0f;
            X.bins.s[a] = (float)h.B / (hi - X.bins.lo[a]);
        }
        for (int l = 0; l < X.L; ++l) X.d[l] = h.d_spec[l];
        X.verts = d.d_vertices;
        X.faces = d.d_faces;
        X.Nv = d.n_vertices;
        X.F = d.n_faces;
        AGAL_TRY(own(bt, &X.coords, (size_t)D * D * X.F));
        AGAL_TRY(own(bt, &X.aabb, (size_t)2 * D * X.F));
        AGAL_TRY(own(bt, &X.rec, (size_t)dev::kRecFloats<D> * X.F));
        AGAL_TRY(own(bt, &X.fidx, (size_t)D * X.F));
        X.bins.B = h.B;
        X.nb = h.nb;
        X.bin_base = bin_base;
        bin_base += h.nb;
        cap_ids += margin(h.P, mg);
        for (int l = 0; l <= X.L; ++l) {
            X.cap[l] = l == 0 ? h.n[0] : margin(h.n[l], mg);
            for (int k = 0; k < (l == 0 ? 1 : 2); ++k) {
                AGAL_TRY(own(bt, &X.keys[l][k], (size_t)X.cap[l]));
                AGAL_TRY(own(bt, &X.leaf[l][k], (size_t)X.cap[l]));
                AGAL_TRY(own(bt, &X.mark[l][k], (size_t)X.cap[l]));
                if (l < X.L) AGAL_TRY(own(bt, &X.cf[l][k], (size_t)X.cap[l] * CELLS));
            }
            if (l == 0) {
                X.keys[0][1] = X.keys[0][0];
                X.leaf[0][1] = X.leaf[0][0];
                X.mark[0][1] = X.mark[0][0];
                X.cf[0][1] = X.cf[0][0];
            }
            if (l < X.L) {
                AGAL_TRY(own(bt, &X.pm[l], (size_t)X.cap[l]));
                AGAL_TRY(own(bt, &X.pos[l], (size_t)X.cap[l] + 1));
                AGAL_TRY(own(bt, &X.mk[l], (size_t)X.cap[l]));
            }
        }
        X.cap_nodes = margin(h.nodes, mg);
        const int64_t nL = X.cap[X.L];
        // list mode as the single-body call takes it, with the face bound taken
        // over extents grown by the margin (a face beyond it is reported)
        const int64_t list_cap = margin(h.list_entries, mg);
        X.lists = h.lists && list_cap <= (int64_t)UINT32_MAX ? 1 : 0;
        if (X.lists) {
            float ext[3];
            for (int a = 0; a < 3; ++a) ext[a] = h.max_extent[a] * (1.0f + mg);
            X.per_face = (int64_t)link_blocks_per_face(D, ext, X.dx[X.L], X.eps);
            X.list_cap = (uint32_t)list_cap;
            X.hash = nullptr;
            X.hmask = 0;
            X.hshift = 0;
            if (X.L > 0) {
                int bits = 6;
                while (bits < 31 && (int64_t(1) << bits) < 2 * ((nL + (1 << D) - 1) >> D)) ++bits;
                X.hmask = (uint32_t)((int64_t(1) << bits) - 1);
                X.hshift = 32 - bits;
                AGAL_TRY(own(bt, &X.hash, (size_t)X.hmask + 1));
            }
            AGAL_TRY(own(bt, &X.nmask, (size_t)nL));
            AGAL_TRY(own(bt, &X.lwork, (size_t)2 * nL));
            AGAL_TRY(own(bt, &X.loff, (size_t)nL + 1));
            AGAL_TRY(own(bt, &X.list, (size_t)list_cap));
            AGAL_TRY(own(bt, &X.lblk, (size_t)list_cap));
            AGAL_TRY(own(bt, &X.nblk, (size_t)X.cap_nodes));
            bt->any_lists = true;
        } else {
            const int64_t stage_rows = kRowCursors * row_range(X.cap_nodes);
            AGAL_TRY(own(bt, &X.skey, (size_t)stage_rows));
            AGAL_TRY(own(bt, &X.sq, (size_t)stage_rows * X.Q));
            AGAL_TRY(own(bt, &X.sface, (size_t)stage_rows * X.Q));
            AGAL_TRY(own(bt, &X.blk_start, (size_t)nL));
        }
        AGAL_TRY(own(bt, &X.blk_count, (size_t)nL));
        AGAL_TRY(own(bt, &X.blk_off, (size_t)nL + 1));
        AGAL_TRY(own(bt, &X.key, (size_t)X.cap_nodes));
        AGAL_TRY(own(bt, &X.q, (size_t)X.cap_nodes * X.Q));
        AGAL_TRY(own(bt, &X.face, (size_t)X.cap_nodes * X.Q));
        if (bt->with_adjoint) {
            AGAL_TRY(own(bt, &X.grad_q, (size_t)X.cap_nodes * X.Q));
            AGAL_TRY(own(bt, &X.grad_v, (size_t)X.Nv * D));
            fill_u32(reinterpret_cast<uint32_t *>(X.grad_q), 0u, X.cap_nodes * X.Q, bt->cap_stream);
        }
    }
    bt->nb_total = bin_base;
    bt->cap_ids = cap_ids;
    // workgroup offsets per body of the kernels laid out body by body; groups: flag passes (kLv), walk q per lattice (3), face-centric flags (1), list build (1), node pass per
    // lattice (3), row pass per lattice (3)
    std::vector<uint32_t> wg_pre((size_t)(kLv + 11) * (bt->nb + 1), 0u);
    for (int b = 0; b < bt->nb; ++b) {
        const BodyDev &X = bt->bodies[b];
        for (int p = 0; p < kLv; ++p) {
            wg_pre[(size_t)p * (bt->nb + 1) + b] = bt->flag_grid[p < agal::kMaxLevels ? p : 0];
            if (p < X.L) bt->flag_grid[p] += (unsigned)((X.cap[p] + (64 / CELLS) - 1) / (64 / CELLS));
        }
        for (int k = 0; k < 3; ++k) {
            const int q = k == 0 ? 9 : (k == 1 ? 19 : 27);
            wg_pre[(size_t)(kLv + k) * (bt->nb + 1) + b] = bt->links_grid[q];
            if (X.Q == q && !X.lists) bt->links_grid[X.Q] += (unsigned)((X.cap[X.L] + (64 / CELLS) - 1) / (64 / CELLS));
            wg_pre[(size_t)(kLv + 5 + k) * (bt->nb + 1) + b] = bt->nodes_grid[q];
            wg_pre[(size_t)(kLv + 8 + k) * (bt->nb + 1) + b] = bt->rows_grid[q];
            if (X.Q == q && X.lists) {
                // node pass: about eight chunks of 64 entries per wave; rows: kRowNodes nodes per wave
                bt->nodes_grid[q] += (unsigned)std::max<int64_t>(1, ((int64_t)X.list_cap + 511) / 512);
                bt->rows_grid[q] += (unsigned)((X.cap_nodes + kRowNodes - 1) / kRowNodes);
            }
        }
        wg_pre[(size_t)(kLv + 4) * (bt->nb + 1) + b] = bt->lfaces_grid;
        if (X.lists) bt->lfaces_grid += (unsigned)((X.F + kLinkFaceG - 1) / kLinkFaceG);
    }
    for (int p = 0; p < kLv; ++p) wg_pre[(size_t)p * (bt->nb + 1) + bt->nb] = bt->flag_grid[p < agal::kMaxLevels ? p : 0];
    // as in the single-body pass: the deduplicating walker when some body's query boxes span more than 64 bins
    // and the pass has fewer than 32 workgroups per CU (bound by its longest waves)
    {
        int ncu = 0, cur = 0;
        if (hipGetDevice(&cur) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, cur) != hipSuccess || ncu < 1)
            ncu = 256;
        (void)hipGetLastError();
        for (int p = 0; p < agal::kMaxLevels; ++p) {
            double most = 0.0;
            for (int b = 0; b < bt->nb; ++b) {
                const BodyDev &X = bt->bodies[b];
                if (X.L <= p) continue;
                double nbins = 1.0;
                for (int a = 0; a < D; ++a)
                    nbins *= std::min((double)X.bins.B, std::floor((4.0 * X.dx[p][a] + 2.0 * X.d[p]) * X.bins.s[a]) + 2.0);
                most = std::max(most, nbins);
            }
            bt->flag_dedup[p] = most > 64.0 && bt->flag_grid[p] < 32u * (unsigned)ncu;
        }
    }
    for (int k = 0; k < 3; ++k) {
        const int q = k == 0 ? 9 : (k == 1 ? 19 : 27);
        wg_pre[(size_t)(kLv + k) * (bt->nb + 1) + bt->nb] = bt->links_grid[q];
        wg_pre[(size_t)(kLv + 5 + k) * (bt->nb + 1) + bt->nb] = bt->nodes_grid[q];
        wg_pre[(size_t)(kLv + 8 + k) * (bt->nb + 1) + bt->nb] = bt->rows_grid[q];
    }
    wg_pre[(size_t)(kLv + 4) * (bt->nb + 1) + bt->nb] = bt->lfaces_grid;
    // face-centric flag step: 4 G faces per workgroup, body by body; a pass takes it when every body refining
    // in it has a block grid within the context's table limit (level 0 needs no table); tables are never
    // cleared (entries are checked against the level's keys)
    {
        int64_t all_faces = 0;
        for (int b = 0; b < bt->nb; ++b) all_faces += bt->bodies[b].F;
        int ncu = 0, cur = 0;
        if (hipGetDevice(&cur) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, cur) != hipSuccess || ncu < 1)
            ncu = 256;
        (void)hipGetLastError();
        bt->fflag_g = face_flag_g(all_faces, ncu);
    }
    const int64_t fper_wg = (int64_t)kFaceFlagWaves * bt->fflag_g;
    for (int b = 0; b < bt->nb; ++b) {
        wg_pre[(size_t)(kLv + 3) * (bt->nb + 1) + b] = bt->fflag_grid;
        bt->fflag_grid += (unsigned)((bt->bodies[b].F + fper_wg - 1) / fper_wg);
    }
    wg_pre[(size_t)(kLv + 3) * (bt->nb + 1) + bt->nb] = bt->fflag_grid;
    for (int p = 0; p < agal::kMaxLevels; ++p) {
        bool ok = p < bt->Lmax;
        for (int b = 0; b < bt->nb && ok; ++b) {
            const BodyDev &X = bt->bodies[b];
            if (X.L <= p) continue;
            int64_t e = 1;
            for (int a = 0; a < D; ++a) e *= (int64_t)X.R[a] << p;
            ok = e <= bt->ctx->flag_table_max &&
                 face_flag_pairs(D, bt->host[b].max_extent, X.d[p], X.dx[p], X.eps) <= kFaceFlagMaxPairs;
        }
        bt->flag_faces[p] = ok;
        if (!ok || p == 0) continue;
        for (int b = 0; b < bt->nb; ++b) {
            BodyDev &X = bt->bodies[b];
            if (X.L <= p) continue;
            int64_t e = 1;
            for (int a = 0; a < D; ++a) e *= (int64_t)X.R[a] << p;
            AGAL_TRY(own(bt, &X.ftable[p], (size_t)e));
        }
    }
    AGAL_TRY(own(bt, &bt->d_wg_pre, wg_pre.size()));
    AGAL_TRY_HIP(hipMemcpyAsync(bt->d_wg_pre, wg_pre.data(), wg_pre.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                bt->cap_stream));
    AGAL_TRY(own(bt, &bt->d_bin_count, (size_t)bt->nb_total));
    AGAL_TRY(own(bt, &bt->d_bin_off, (size_t)bt->nb_total + 1));
    AGAL_TRY(own(bt, &bt->d_bin_cursor, (size_t)bt->nb_total));
    AGAL_TRY(own(bt, &bt->d_ids, (size_t)cap_ids));
    AGAL_TRY(own(bt, &bt->d_big, (size_t)(cap_ids / 2048 + 2)));
    AGAL_TRY(own(bt, &bt->d_med, (size_t)bt->nb_total + 1));
    for (int b = 0; b < bt->nb; ++b) {
        bt->bodies[b].bins.off = bt->d_bin_off + bt->bodies[b].bin_base;
        bt->bodies[b].bins.ids = bt->d_ids;
    }
    AGAL_TRY(own(bt, &bt->d_cnt, (size_t)bt->nb * kLv));
    AGAL_TRY(own(bt, &bt->d_nodes, (size_t)bt->nb));
    AGAL_TRY(own(bt, &bt->d_cursor, (size_t)bt->nb * kRowCursors * kCursorStride));
    AGAL_TRY(own(bt, &bt->d_ctl, 1));
    AGAL_TRY(own(bt, &bt->d_bodies, (size_t)bt->nb));

    // ---- scan segments and their status scratch ------------------------------
    auto tiles = [](int64_t cap) { return (cap + kScanTile) / kScanTile; };
    int64_t sw = 0;
    auto add_seg = [&](const void *in, uint32_t *out, const uint32_t *n_dev, int64_t n_const, int64_t cap) {
        Seg sg{in, out, n_dev, n_const, sw};
        bt->seg_store.push_back(sg);
        sw += tiles(cap);
    };
    int64_t max_sw = 0;
    bt->bins_seg_off = (int)bt->seg_store.size();
    add_seg(bt->d_bin_count, bt->d_bin_off, nullptr, bt->nb_total, bt->nb_total);
    max_sw = std::max(max_sw, sw);
    for (int p = 0; p < bt->Lmax; ++p) {
        sw = 0;
        bt->pass_seg_off.push_back((int)bt->seg_store.size());
        for (int b = 0; b < bt->nb; ++b)
            for (int m = 0; m <= p; ++m) {
                const BodyDev &X = bt->bodies[b];
                if (X.L > p) add_seg(X.pm[m], X.pos[m], bt->d_cnt + b * kLv + m, 0, X.cap[m]);
                else add_seg(nullptr, nullptr, nullptr, 0, 0);   // placeholder keeps (b, m) indexing
            }
        bt->pass_seg_n.push_back(bt->nb * (p + 1));
        max_sw = std::max(max_sw, sw);
    }
    sw = 0;
    bt->links_seg_off = (int)bt->seg_store.size();
    for (int b = 0; b < bt->nb; ++b) {
        const BodyDev &X = bt->bodies[b];
        add_seg(X.blk_count, X.blk_off, bt->d_cnt + b * kLv + X.L, 0, X.cap[X.L]);
    }
    max_sw = std::max(max_sw, sw);
    sw = 0;
    bt->lists_seg_off = (int)bt->seg_store.size();
    for (int b = 0; b < bt->nb; ++b) {
        const BodyDev &X = bt->bodies[b];
        if (X.lists) add_seg(X.lwork, X.loff, bt->d_cnt + b * kLv + X.L, 0, X.cap[X.L]);
        else add_seg(nullptr, nullptr, nullptr, 0, 0);
    }
    max_sw = std::max(max_sw, sw);
    // placeholders of finished bodies must not be scanned: give them n = 0 and a
    // harmless output word
    uint32_t *dummy = nullptr;
    AGAL_TRY(own(bt, &dummy, 4));
    for (auto &sg : bt->seg_store)
        if (!sg.out) {
            sg.out = dummy;
            sg.in = dummy;
            sg.n_const = 0;
            sg.n_dev = nullptr;
        }
    bt->status_words = max_sw + 1;
    const int n_scans = bt->Lmax + 3;   // bins, one per pass, links, candidate lists
    AGAL_TRY(own(bt, &bt->d_status, (size_t)bt->status_words * n_scans));
    AGAL_TRY(own(bt, &bt->d_tickets, (size_t)n_scans));
    AGAL_TRY(own(bt, &bt->d_segpre, (size_t)n_scans * (kMaxSeg + 1)));
    AGAL_TRY(own(bt, &bt->d_segs, bt->seg_store.size()));

    // ---- fill table: everything a run needs cleared, in the run's first launch --
    std::vector<Fill> fills;
    auto words = [](size_t bytes) { return (int64_t)((bytes + 3) / 4); };
    fills.push_back({bt->d_bin_count, words(bt->nb_total * 4), 0u});
    fills.push_back({bt->d_bin_cursor, words(bt->nb_total * 4), 0u});
    fills.push_back({reinterpret_cast<uint32_t *>(bt->d_status), words((size_t)bt->status_words * n_scans * 8), 0u});
    fills.push_back({bt->d_tickets, n_scans, 0u});
    for (int b = 0; b < bt->nb; ++b) {
        const BodyDev &X = bt->bodies[b];
        for (int m = 0; m < X.L; ++m) fills.push_back({reinterpret_cast<uint32_t *>(X.pm[m]), words(X.cap[m]), 0u});
        if (bt->with_adjoint)
            fills.push_back({reinterpret_cast<uint32_t *>(X.grad_v), words(X.Nv * D * 4), 0u});
        if (X.lists) {
            if (X.hash) fills.push_back({reinterpret_cast<uint32_t *>(X.hash), 2 * ((int64_t)X.hmask + 1), ~0u});
            fills.push_back({X.lwork, 2 * X.cap[X.L], 0u});
        }
    }
    bt->n_fill_init = (int)fills.size();
    AGAL_TRY(own(bt, &bt->d_fills, fills.size()));
    AGAL_TRY_HIP(hipMemcpyAsync(bt->d_fills, fills.data(), fills.size() * sizeof(Fill), hipMemcpyHostToDevice,
                                bt->cap_stream));
    AGAL_TRY_HIP(hipMemcpyAsync(bt->d_segs, bt->seg_store.data(), bt->seg_store.size() * sizeof(Seg),
                                hipMemcpyHostToDevice, bt->cap_stream));
    AGAL_TRY_HIP(hipMemcpyAsync(bt->d_bodies, bt->bodies.data(), bt->nb * sizeof(BodyDev), hipMemcpyHostToDevice,
                                bt->cap_stream));
    AGAL_TRY_HIP(hipStreamSynchronize(bt->cap_stream));

    // ---- capture (and pick the persistent grid) -------------------------------
    int dev = 0;
    AGAL_TRY_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    AGAL_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    bt->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (opt.tune_grid) {
        double best = 1e30;
        int bestw = 4;
        for (int w : {1, 2, 4, 8}) {
            bt->wg_per_cu = w;
            AGAL_TRY(capture<D>(bt));
            double ms = 0;
            AGAL_TRY(time_graph(bt, 3, &ms));
            if (ms < best) {
                best = ms;
                bestw = w;
            }
        }
        bt->wg_per_cu = bestw;
    }
    AGAL_TRY(capture<D>(bt));
    return AGAL_OK;
}

}  // namespace batch
}  // namespace agal

using namespace agal;

extern "C" {

agal_status agal_batch_plan_create(agal_context ctx, int n_bodies, const agal_body_desc *bodies,
                                   const agal_tune_opts *opts, void *stream, agal_batch *out) {
    if (!ctx || !bodies || !out) return fail(AGAL_EINVAL, "agal_batch_plan_create: NULL argument");
    if (n_bodies < 1 || n_bodies > batch::kMaxBodies)
        return fail(AGAL_EINVAL, "agal_batch_plan_create: n_bodies must be in [1, %d]", batch::kMaxBodies);
    const int D = bodies[0].dim;
    for (int b = 0; b < n_bodies; ++b) {
        const agal_body_desc &d = bodies[b];
        if (d.dim != D || d.forest.dim != D)
            return fail(AGAL_EINVAL, "agal_batch_plan_create: body %d: every body needs dim %d", b, D);
        agal::Lattice lat;
        if (!lattice_table(d.lattice, &lat) || lat.dim != D)
            return fail(AGAL_EINVAL, "agal_batch_plan_create: body %d: lattice does not match the dimension", b);
        if (d.forest.n_levels < 0 || d.forest.n_levels > kMaxLevels)
            return fail(AGAL_EINVAL, "agal_batch_plan_create: body %d: n_levels outside [0, %d]", b, kMaxLevels);
        if (d.forest.n_levels > 0 && !d.forest.d_spec)
            return fail(AGAL_EINVAL, "agal_batch_plan_create: body %d: d_spec is NULL", b);
    }
    agal_tune_opts opt{};
    if (opts) opt = *opts;
    auto *bt = new (std::nothrow) agal_batch_t();
    if (!bt) return fail(AGAL_ENOMEM, "agal_batch_plan_create: host allocation failed");
    bt->ctx = ctx;
    bt->nb = n_bodies;
    bt->dim = D;
    bt->with_adjoint = opt.with_adjoint != 0;
    bt->host.resize(n_bodies);
    for (int b = 0; b < n_bodies; ++b) {
        bt->host[b].desc = bodies[b];
        bt->host[b].d_spec.assign(bodies[b].forest.d_spec, bodies[b].forest.d_spec + bodies[b].forest.n_levels);
        bt->host[b].desc.forest.d_spec = bt->host[b].d_spec.data();
    }
    hipError_t e = hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete bt;
        return fail(AGAL_EHIP, "agal_batch_plan_create: hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    agal_status st = D == 3 ? batch::plan<3>(bt, opt, (hipStream_t)stream) : batch::plan<2>(bt, opt, (hipStream_t)stream);
    if (st != AGAL_OK) {
        agal_destroy_batch(bt);
        return st;
    }
    *out = bt;
    return AGAL_OK;
}

agal_status agal_batch_run(agal_batch b, void *stream) {
    if (!b || !b->exec) return fail(AGAL_EINVAL, "agal_batch_run: no plan");
    hipStream_t s = (hipStream_t)stream;
    {
        ProfScope prof(b->ctx, "batch_graph", s);
        AGAL_TRY_HIP(hipGraphLaunch(b->exec, s));
    }
    b->have_status = false;
    return AGAL_OK;
}

agal_status agal_batch_status(agal_batch b, void *stream) {
    if (!b) return fail(AGAL_EINVAL, "agal_batch_status: NULL batch");
    hipStream_t s = (hipStream_t)stream;
    b->h_cnt.assign((size_t)b->nb * batch::kLv, 0);
    b->h_nodes.assign((size_t)b->nb, 0);
    batch::Ctl ctl{};
    AGAL_TRY_HIP(hipMemcpyAsync(b->h_cnt.data(), b->d_cnt, b->h_cnt.size() * 4, hipMemcpyDeviceToHost, s));
    AGAL_TRY_HIP(hipMemcpyAsync(b->h_nodes.data(), b->d_nodes, b->h_nodes.size() * 4, hipMemcpyDeviceToHost, s));
    AGAL_TRY_HIP(hipMemcpyAsync(&ctl, b->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, s));
    AGAL_TRY_HIP(hipStreamSynchronize(s));
    b->h_overflow = ctl.overflow;
    b->h_err = ctl.err;
    b->have_status = true;
    if (ctl.err) return fail(AGAL_EINVAL, "agal_batch_status: invalid input (bit 0: non-finite coordinate, "
                                         "bit 1: vertex index out of range): %u", ctl.err);
    if (ctl.overflow)
        return fail(AGAL_ECAPACITY, "agal_batch_status: capacity exceeded (bit 0: bins, bit 1: forest level, "
                                    "bit 2: nodes, bit 3: candidate lists): %u", ctl.overflow);
    if (ctl.balance) return fail(AGAL_ESTATE, "agal_batch_status: a forest lost 2:1 balance");
    return AGAL_OK;
}

agal_status agal_batch_body_view(agal_batch b, int body, const uint64_t **d_node_key, const float **d_q,
                                 const int32_t **d_face, int64_t *n_nodes, int *Q, float **d_grad_q,
                                 const float **d_grad_vertices, int64_t *node_capacity, int32_t *bins) {
    if (!b) return fail(AGAL_EINVAL, "agal_batch_body_view: NULL batch");
    if (body < 0 || body >= b->nb) return fail(AGAL_EINVAL, "agal_batch_body_view: body %d out of range", body);
    const auto &X = b->bodies[body];
    if (d_node_key) *d_node_key = X.key;
    if (d_q) *d_q = X.q;
    if (d_face) *d_face = X.face;
    if (n_nodes) *n_nodes = b->have_status ? b->h_nodes[body] : -1;
    if (Q) *Q = X.Q;
    if (d_grad_q) *d_grad_q = X.grad_q;
    if (d_grad_vertices) *d_grad_vertices = X.grad_v;
    if (node_capacity) *node_capacity = X.cap_nodes;
    if (bins) *bins = b->host[body].B;
    return AGAL_OK;
}

agal_status agal_batch_level_view(agal_batch b, int body, int level, const uint32_t **d_keys, const uint8_t **d_leaf,
                                  const uint8_t **d_mark, const uint8_t **d_cell_flag, int64_t *n_blocks) {
    if (!b) return fail(AGAL_EINVAL, "agal_batch_level_view: NULL batch");
    if (body < 0 || body >= b->nb) return fail(AGAL_EINVAL, "agal_batch_level_view: body %d out of range", body);
    const auto &X = b->bodies[body];
    if (level < 0 || level > X.L) return fail(AGAL_EINVAL, "agal_batch_level_view: level %d outside [0, %d]", level, X.L);
    const int k = level == 0 ? 0 : ((X.L - level) & 1);
    if (d_keys) *d_keys = X.keys[level][k];
    if (d_leaf) *d_leaf = X.leaf[level][k];
    if (d_mark) *d_mark = X.mark[level][k];
    if (d_cell_flag) *d_cell_flag = level < X.L ? X.cf[level][k] : nullptr;
    if (n_blocks) *n_blocks = b->have_status ? b->h_cnt[(size_t)body * batch::kLv + level] : -1;
    return AGAL_OK;
}

agal_status agal_batch_info(agal_batch b, int *n_bodies, int *workgroups_per_cu) {
    if (!b) return fail(AGAL_EINVAL, "agal_batch_info: NULL batch");
    if (n_bodies) *n_bodies = b->nb;
    if (workgroups_per_cu) *workgroups_per_cu = b->wg_per_cu;
    return AGAL_OK;
}

void agal_destroy_batch(agal_batch b) {
    if (!b) return;
    if (b->cap_stream) (void)hipStreamSynchronize(b->cap_stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *p : b->owned) b->ctx->mem.release(p, b->cap_stream);
    if (b->cap_stream) {
        (void)hipStreamSynchronize(b->cap_stream);
        (void)hipStreamDestroy(b->cap_stream);
    }
    delete b;
}

}  // extern "C"
