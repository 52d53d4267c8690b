// Per-item device code of every kernel of the path: one wave's blocks for the
// flag and link kernels, one thread's item for the balance and merge steps,
// one workgroup's node tile for the adjoint, one face / bin group for the
// binning.  The single-body kernels (refine.hip, links.hip, bins.hip) and the
// batched persistent kernels (batch.hip) are thin loops around these, so both
// forms compute bit-identical flags and link fractions.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>
#include <climits>

#include "device.hpp"

namespace agal {
namespace kern {

// ===========================================================================
// Import (paper Sec. II-B)
// ===========================================================================
// Face f: validate its indices, gather its corners into the structure-of-arrays
// coordinate list, the bounding-box rows and the per-face record, and copy
// its indices.  Returns error bits: 2 for an index outside [0, Nv) (the face
// is then written as zeros).
template <int D>
__device__ __forceinline__ uint32_t import_face(const float *verts, int64_t Nv, const int32_t *faces, int64_t F,
                                                float *coords, float *aabb, float *rec, int32_t *fidx, int64_t f,
                                                float *ext = nullptr) {
    float v[D][D];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int64_t vi = faces ? (int64_t)faces[f * D + k] : f * D + k;
        ok = ok && vi >= 0 && vi < Nv;
        fidx[f * D + k] = (vi >= 0 && vi < Nv) ? (int32_t)vi : 0;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int64_t vi = faces ? (int64_t)faces[f * D + k] : f * D + k;
#pragma unroll
        for (int a = 0; a < D; ++a) v[k][a] = ok ? verts[vi * D + a] : 0.0f;
    }
    float r[dev::kRecFloats<D>];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int a = 0; a < D; ++a) {
            coords[(int64_t)(k * D + a) * F + f] = v[k][a];
            r[k * D + a] = v[k][a];
        }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        float mn = v[0][a], mx = v[0][a];
#pragma unroll
        for (int k = 1; k < D; ++k) {
            mn = dev::fminf_(mn, v[k][a]);
            mx = dev::fmaxf_(mx, v[k][a]);
        }
        aabb[(int64_t)a * F + f] = mn;
        aabb[(int64_t)(D + a) * F + f] = mx;
        r[D * D + a] = mn;
        r[D * D + D + a] = mx;
        if (ext) ext[a] = fmaxf(ext[a], mx - mn);   // largest box extent per axis (NaN ignored)
    }
    if constexpr (D == 3) r[15] = 0.0f;
    float4 *out = reinterpret_cast<float4 *>(rec) + f * (dev::kRecFloats<D> / 4);
#pragma unroll
    for (int i = 0; i < dev::kRecFloats<D> / 4; ++i)
        out[i] = make_float4(r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3]);
    return ok ? 0u : 2u;
}

// ===========================================================================
// Spatial binning (paper Sec. II-C-3)
// ===========================================================================
constexpr int kCanonCap = 2048;      // ids per LDS segment in the rank sort
constexpr int kBigThreads = 1024;

template <int D>
__device__ __forceinline__ void face_bin_range(const float *aabb, int64_t F, int64_t f, const dev::BinGrid &g,
                                               int lo[3], int hi[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) { lo[a] = 0; hi[a] = 0; }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        lo[a] = dev::bin_of(aabb[(int64_t)a * F + f], g.lo[a], g.s[a], g.B);
        hi[a] = dev::bin_of(aabb[(int64_t)(D + a) * F + f], g.lo[a], g.s[a], g.B);
    }
}

// atomicAdd(p, 1) for every active lane, returning its old value, with the
// lanes whose counter is the first active lane's combined into one atomic (up
// to four such rounds; the rest add alone).  With few bins many faces of a
// wave share one, and same-address atomics from every face would serialise.
// Lanes are matched by address, so lanes of different arrays never combine.
// Slots of combined lanes follow the lane order.
__device__ __forceinline__ uint32_t add_one_combined(uint32_t *p) {
    const int lane = dev::lane_id();
    const uint64_t a = (uint64_t)(uintptr_t)p;
    bool pending = true;
    uint32_t slot = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t act = __ballot(pending);
        if (!act) break;
        const int leader = __builtin_ctzll(act);
        const uint64_t la = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(a >> 32), leader) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)a, leader);
        const bool mine = pending && a == la;
        const uint64_t m = __ballot(mine);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(p, (uint32_t)__popcll(m));
        base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
        if (mine) {
            slot = base + (uint32_t)dev::lanes_below(m);
            pending = false;
        }
    }
    if (pending) slot = atomicAdd(p, 1u);
    return slot;
}

template <int D>
__device__ __forceinline__ void bin_count_item(const float *aabb, int64_t F, const dev::BinGrid &g, uint32_t *count,
                                               int64_t f) {
    {
        int lo[3], hi[3];
        face_bin_range<D>(aabb, F, f, g, lo, hi);
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x)
                    (void)add_one_combined(count + ((int64_t)z * g.B + y) * g.B + x);
    }
}

template <int D>
__device__ __forceinline__ void bin_scatter_item(const float *aabb, int64_t F, const dev::BinGrid &g,
                                                 const uint32_t *off, uint32_t *cursor, int32_t *ids, int64_t f) {
    {
        int lo[3], hi[3];
        face_bin_range<D>(aabb, F, f, g, lo, hi);
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    int64_t b = ((int64_t)z * g.B + y) * g.B + x;
                    uint32_t pos = off[b] + add_one_combined(cursor + b);
                    ids[pos] = (int32_t)f;
                }
    }
}

// Sort ids[s0, s1) (bins b_first..b_last whose offsets are in s_off) by rank:
// each entry's position inside its bin is the number of smaller ids there.
__device__ void rank_sort_segment(int32_t *ids, const uint32_t *s_off, int nbins, uint32_t s0, uint32_t s1,
                                  int32_t *s_val) {
    const int lane = threadIdx.x;
    const int n = (int)(s1 - s0);
    for (int e = lane; e < n; e += dev::kWave) s_val[e] = ids[s0 + e];
    __syncthreads();
    for (int e = lane; e < n; e += dev::kWave) {
        uint32_t pos = s0 + (uint32_t)e;
        // bin of entry e: last bin whose start <= pos
        int lo = 0, hi = nbins - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= pos) lo = mid; else hi = mid - 1;
        }
        // the last bin starting at or before pos is the non-empty one holding it
        int b = lo;
        const int bs = (int)(s_off[b] - s0), be = (int)(s_off[b + 1] - s0);
        const int32_t v = s_val[e];
        int rank = 0;
        for (int j = bs; j < be; ++j) rank += s_val[j] < v ? 1 : 0;
        ids[s0 + bs + rank] = v;
    }
    __syncthreads();
}

// One wave: the group of 64 consecutive bins starting at b0.  A group whose
// ids fit the LDS segment is rank-sorted here in one go; otherwise each of
// its bins with more than one id goes to a list of its own: the medium list
// (at most kCanonCap ids: rank-sorted by a workgroup per bin) or, tagged with
// big_tag, the big list (rebuilt by an ordered sweep).  Lists are appended
// through counters (lists[0], lists[1] = medium and big counts).
__device__ __forceinline__ void bin_canon_group(int32_t *ids, const uint32_t *off, int64_t nb, int64_t b0,
                                                uint32_t *med_list, uint32_t *big_list, uint32_t *counts,
                                                uint32_t big_tag) {
    __shared__ uint32_t s_off[dev::kWave + 1];
    __shared__ int32_t s_val[kCanonCap];
    const int nbins = (int)std::min<int64_t>(dev::kWave, nb - b0);
    const int lane = threadIdx.x;
    for (int i = lane; i <= nbins; i += dev::kWave) s_off[i] = off[b0 + i];
    __syncthreads();
    const uint32_t g0 = s_off[0], g1 = s_off[nbins];
    if (g1 - g0 <= 1) {
        __syncthreads();
        return;
    }
    if (g1 - g0 <= (uint32_t)kCanonCap) {
        rank_sort_segment(ids, s_off, nbins, g0, g1, s_val);
        return;
    }
    // group too large: each bin on its own (one lane per bin of the group)
    if (lane < nbins) {
        const uint32_t a0 = s_off[lane], a1 = s_off[lane + 1];
        if (a1 - a0 > (uint32_t)kCanonCap) big_list[atomicAdd(counts + 1, 1u)] = big_tag + (uint32_t)(b0 + lane);
        else if (a1 - a0 > 1) med_list[atomicAdd(counts, 1u)] = (uint32_t)(b0 + lane);
    }
    __syncthreads();
}

// One workgroup of kMedThreads threads: bin b's segment (at most kCanonCap
// ids) sorted by rank in LDS.
constexpr int kMedThreads = 256;
__device__ __forceinline__ void bin_canon_medium(int32_t *ids, const uint32_t *off, int64_t b) {
    __shared__ int32_t s_val[kCanonCap];
    const uint32_t s0 = off[b], s1 = off[b + 1];
    const int n = (int)(s1 - s0);
    for (int e = threadIdx.x; e < n; e += kMedThreads) s_val[e] = ids[s0 + e];
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += kMedThreads) {
        const int32_t v = s_val[e];
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += s_val[j] < v ? 1 : 0;
        ids[s0 + rank] = v;
    }
    __syncthreads();
}

// Bins with more than kCanonCap ids: rewrite the segment by an ordered sweep
// over all faces (membership recomputed from the bounding boxes).
// One workgroup of kBigThreads threads rebuilds bin b's segment.
template <int D>
__device__ __forceinline__ void bin_canon_big_bin(const float *aabb, int64_t F, const dev::BinGrid &g,
                                                  const uint32_t *off, int32_t *ids, int64_t b) {
    __shared__ uint32_t s_wsum[kBigThreads / dev::kWave];
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x % dev::kWave;
    {
        const int bx = (int)(b % g.B);
        const int by = (int)((b / g.B) % g.B);
        const int bz = D == 3 ? (int)(b / ((int64_t)g.B * g.B)) : 0;
        uint32_t run = off[b];
        for (int64_t f0 = 0; f0 < F; f0 += kBigThreads) {
            const int64_t f = f0 + threadIdx.x;
            uint32_t mem = 0;
            if (f < F) {
                int lo[3], hi[3];
                face_bin_range<D>(aabb, F, f, g, lo, hi);
                mem = (bx >= lo[0] && bx <= hi[0] && by >= lo[1] && by <= hi[1] && bz >= lo[2] && bz <= hi[2]) ? 1u : 0u;
            }
            uint32_t incl = dev::wave_inclusive_sum(mem);
            if (lane == dev::kWave - 1) s_wsum[w] = incl;
            __syncthreads();
            uint32_t pre = 0, tot = 0;
            for (int j = 0; j < kBigThreads / dev::kWave; ++j) {
                if (j < w) pre += s_wsum[j];
                tot += s_wsum[j];
            }
            if (mem) ids[run + pre + incl - 1] = (int32_t)f;
            run += tot;
            __syncthreads();
        }
    }
}


// ===========================================================================
// Candidate faces of a box (shared by the flag and q kernels)
// ===========================================================================
// Walks the face ids of bins [ilo, ihi] (inclusive, per axis) in rounds of 64,
// one candidate per lane: round(has, f, cur) is called by the whole wave, with
// `cur` the bin coordinates of the lane's candidate, and returns false to stop.
// Up to 64 bins are opened at once (one lane per bin, offsets loaded together;
// a wave prefix of their sizes makes one list), so small bins share rounds,
// and the ids of the next round are loaded while the current round runs:
// about one memory latency per 64 candidates instead of two per bin.
template <class Round>
__device__ __forceinline__ void for_candidates(const dev::BinGrid &g, const int ilo[3], const int ihi[3],
                                               Round &&round) {
    const int lane = dev::lane_id();
    const int nx = ihi[0] - ilo[0] + 1, ny = ihi[1] - ilo[1] + 1, nz = ihi[2] - ilo[2] + 1;
    const int nbins = nx * ny * nz;
    for (int bg = 0; bg < nbins; bg += dev::kWave) {
        const int bi = bg + lane;
        uint32_t s0 = 0, cnt = 0;
        if (bi < nbins) {
            const int bx = ilo[0] + bi % nx, by = ilo[1] + (bi / nx) % ny, bz = ilo[2] + bi / (nx * ny);
            const int64_t b = ((int64_t)bz * g.B + by) * g.B + bx;
            s0 = g.off[b];
            cnt = g.off[b + 1] - s0;
        }
        const uint32_t incl = dev::wave_inclusive_sum(cnt);
        const uint32_t pre = incl - cnt;
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, dev::kWave - 1);   // scalar
        const uint64_t nonempty = __ballot(cnt > 0);
        // id of list entry c0 + lane (or -1) and the lane holding its bin.  The
        // cross-lane reads run with every lane active: a lane reading from an
        // inactive lane gets 0, not that lane's value.
        auto fetch = [&](uint32_t c0, int &k) -> int32_t {
            const uint32_t v = c0 + lane;
            k = 0;
            for (uint64_t m = nonempty; m; m &= m - 1ull) {
                const int kk = __builtin_ctzll(m);
                k = __builtin_amdgcn_readlane(pre, kk) <= v ? kk : k;
            }
            const uint32_t s0k = __shfl(s0, k, dev::kWave);
            const uint32_t prek = __shfl(pre, k, dev::kWave);
            if (v >= total) return -1;
            const int32_t id = g.ids[s0k + (v - prek)];
            return id >= 0 && (int64_t)id < g.F ? id : -1;
        };
        int k = 0;
        int32_t f = fetch(0, k);
        for (uint32_t c0 = 0; c0 < total; c0 += dev::kWave) {
            int kn = 0;
            const int32_t fn = c0 + dev::kWave < total ? fetch(c0 + dev::kWave, kn) : -1;   // next round, in flight
            const int bk = bg + k;
            const int cur[3] = {ilo[0] + bk % nx, ilo[1] + (bk / nx) % ny, ilo[2] + bk / (nx * ny)};
            if (!round(f >= 0, f, cur)) return;
            f = fn;
            k = kn;
        }
    }
}

// Each face of bins [ilo, ihi] once, for boxes that span many bins (the flag
// pass): ids are read four rounds of 64 at a time (one memory latency per 256
// list entries), an LDS hash set of face ids drops the repeats of a face that
// lies in several bins, and the records of the faces that remain are loaded
// 64 at a time.  stage(has, f, r) is called by the whole wave with up to 64
// such faces (r the lane's face record) and returns false to stop.  A face
// that finds no free slot within kSeenProbes tries is passed on as new, so a
// crowded set can let a repeat through; stage() must tolerate that.
constexpr int kSeen = 1024;             // hash-set slots (power of two)
constexpr int kSeenProbes = 16;         // slots tried before a face is let through as new
constexpr int kUniqCap = 5 * 64;        // faces waiting for their records

template <int D, class Stage>
__device__ __forceinline__ void for_unique_candidates(const dev::BinGrid &g, const float *rec, const int ilo[3],
                                                      const int ihi[3], int32_t *s_seen, int32_t *s_list,
                                                      uint32_t *s_bpre, uint32_t *s_bs0, Stage &&stage) {
    constexpr int RF = dev::kRecFloats<D>;
    const int lane = dev::lane_id();
    const int nx = ihi[0] - ilo[0] + 1, ny = ihi[1] - ilo[1] + 1, nz = ihi[2] - ilo[2] + 1;
    const int nbins = nx * ny * nz;
    __syncthreads();
    for (int i = lane; i < kSeen; i += dev::kWave) s_seen[i] = -1;
    int nl = 0;   // wave-uniform list length
    // records of list entries 0 .. t-1, one per lane, to stage(); the rest moves to the front
    auto flush = [&](int t) -> bool {
        __syncthreads();
        const int32_t f = lane < t ? s_list[lane] : -1;
        __syncthreads();
        for (int i = lane; i < nl - t; i += dev::kWave) s_list[i] = s_list[t + i];   // up to 4 x 64 remain
        nl -= t;
        float r[RF];
        if (f >= 0) dev::load_rec<D>(rec, f, r);
        return stage(f >= 0, f, (const float *)r);
    };
    for (int bg = 0; bg < nbins; bg += dev::kWave) {
        const int bi = bg + lane;
        uint32_t s0 = 0, cnt = 0;
        if (bi < nbins) {
            const int bx = ilo[0] + bi % nx, by = ilo[1] + (bi / nx) % ny, bz = ilo[2] + bi / (nx * ny);
            const int64_t b = ((int64_t)bz * g.B + by) * g.B + bx;
            s0 = g.off[b];
            cnt = g.off[b + 1] - s0;
        }
        const uint32_t incl = dev::wave_inclusive_sum(cnt);
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, dev::kWave - 1);   // scalar
        if (total == 0) continue;
        // the non-empty bins in list order, for a binary search per list entry
        const uint64_t ne = __ballot(cnt > 0);
        const int nne = __popcll(ne);
        __syncthreads();
        if (cnt > 0) {
            const int k = dev::lanes_below(ne);
            s_bpre[k] = incl - cnt;
            s_bs0[k] = s0;
        }
        __syncthreads();
        for (uint32_t c0 = 0; c0 < total; c0 += 4 * dev::kWave) {
            int32_t id[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t v = c0 + q * dev::kWave + lane;
                id[q] = -1;
                if (v < total) {
                    int lo = 0, hi = nne - 1;   // last non-empty bin starting at or before v
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_bpre[mid] <= v) lo = mid;
                        else hi = mid - 1;
                    }
                    const int32_t f = g.ids[s_bs0[lo] + (v - s_bpre[lo])];
                    id[q] = f >= 0 && (int64_t)f < g.F ? f : -1;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                bool fresh = false;
                if (id[q] >= 0) {
                    uint32_t h = ((uint32_t)id[q] * 2654435761u) >> 22;   // 10 bits: kSeen slots
                    fresh = true;   // a crowded set lets the face through
                    for (int probe = 0; probe < kSeenProbes; ++probe) {
                        const int32_t prev = atomicCAS(&s_seen[h], -1, id[q]);
                        if (prev == -1) break;
                        if (prev == id[q]) {
                            fresh = false;
                            break;
                        }
                        h = (h + 1) & (kSeen - 1);
                    }
                }
                const uint64_t m = __ballot(fresh);
                if (fresh) s_list[nl + dev::lanes_below(m)] = id[q];
                nl += __popcll(m);
            }
            while (nl >= dev::kWave)
                if (!flush(dev::kWave)) return;
        }
    }
    if (nl > 0) (void)flush(nl);
}

// ===========================================================================
// Near-wall refinement (paper Sec. II-C-1, II-C-2)
// ===========================================================================
constexpr int kFlagCap = 128;  // staged candidate faces per wave

template <int D>
struct FlagArgs {
    dev::Faces faces;
    dev::BinGrid bins;
    const uint32_t *keys;
    int64_t n;
    int level;
    int R[3];
    float lo[3];
    float dx[3];
    float eps[3];
    float h;
    uint8_t *cf;     // n * 4^D
    uint8_t *pmark;  // n
};

// One wave: blocks first .. first + 64/4^D - 1 of A (one lane per cell).
template <int D, bool kDedup = false>
__device__ __forceinline__ void flag_wave(const FlagArgs<D> &A, int64_t first) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int BPW = 64 / CELLS;
    constexpr int NF = D * D;   // staged corner coordinates
    __shared__ float s_f[NF][kFlagCap];
    __shared__ __align__(16) uint32_t s_code[kFlagCap];
    const int lane = threadIdx.x;
    const int64_t blk = first + lane / CELLS;
    const bool valid = blk < A.n;
    const int cell = lane % CELLS;
    const int sub = lane / CELLS;

    int bc[3] = {0, 0, 0};
    if (valid) dev::decode_key<D>(A.keys[blk], A.level, A.R[0], A.R[1], bc);
    const int pos3[3] = {cell & 3, (cell >> 2) & 3, cell >> 4};
    float m[3];
    m[0] = dev::cell_centre(A.lo[0], 4 * bc[0] + pos3[0], A.dx[0]);
    m[1] = dev::cell_centre(A.lo[1], 4 * bc[1] + pos3[1], A.dx[1]);
    m[2] = D == 3 ? dev::cell_centre(A.lo[2], 4 * bc[2] + pos3[2], A.dx[2]) : 0.0f;
    const float h = A.h;
    bool flagged = !valid;

    // The box-axis part of the separating-axis test is separable: cell (i0,i1,i2)
    // of a block is not separated from a face along axis a exactly when position
    // i_a passes the axis-a test, so a staged face carries one bit per (axis,
    // position) of the block it was staged for, computed with the same FP32
    // expressions every lane would use (min_k fl(v_k - m) = fl(min_k v_k - m)),
    // and a lane tests a face with one AND against its own D bits.  (In 2D the
    // four blocks of a wave take bits 8t..8t+7; a face near a cell of block t
    // lies in block t's query box, so it is staged, and coded, for block t.)
    uint32_t lbits = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) lbits |= 1u << (sub * 4 * D + 4 * a + pos3[a]);
    float mc[D][4];   // cell centres along each axis of the block being staged
    auto face_code = [&](int t, const float *bb) -> uint32_t {   // bb: min[D], max[D]
        uint32_t c = 0;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float lo_a = bb[a] - mc[a][i], hi_a = bb[D + a] - mc[a][i];
                c |= (!(lo_a > h) && !(hi_a < -h)) ? (1u << (4 * a + i)) : 0u;
            }
        return c << (t * 4 * D);
    };

    int count = 0;  // staged faces (wave-uniform)
    // The full tests wait in a queue of (lane, staged face) pairs and are taken
    // 64 at a time, one per lane, whichever lane queued them: a cell near many
    // faces does not hold the wave while the other lanes idle.  A pair whose
    // cell is flagged meanwhile is dropped.
    constexpr int TCAP = 128;   // below 64 after a take, at most 64 added per step
    __shared__ uint32_t s_q[TCAP];
    __shared__ float s_m[64][3];
    __shared__ int s_fl[64];
#pragma unroll
    for (int a = 0; a < 3; ++a) s_m[lane][a] = m[a];
    s_fl[lane] = flagged ? 1 : 0;
    int nq = 0;   // wave-uniform
    auto take = [&](int t) {
        __syncthreads();
        const uint32_t item = lane < t ? s_q[lane] : 0u;
        __syncthreads();
        if (lane < nq - t) s_q[lane] = s_q[t + lane];
        nq -= t;
        const int l = (int)(item >> 7), j = (int)(item & 127u);
        if (lane < t && !s_fl[l]) {
            float v[D * D];
#pragma unroll
            for (int k = 0; k < D * D; ++k) v[k] = s_f[k][j];
            const float ml[3] = {s_m[l][0], s_m[l][1], s_m[l][2]};
            bool hit;
            if constexpr (D == 3) hit = dev::sat_triangle(v, ml, h);
            else hit = dev::sat_segment(v, ml, h);
            if (hit) s_fl[l] = 1;
        }
    };
    // Batches of 64 staged faces: each lane marks the faces its cube's box axes do
    // not separate from it and queues them for the full test, until flagged.
    auto test_staged = [&](int n) {
        __syncthreads();
        for (int j0 = 0; j0 < n; j0 += 64) {
            flagged = s_fl[lane] != 0;
            if (__ballot(!flagged) == 0) break;
            const int jn = min(64, n - j0);
            uint64_t nm = 0;
            if (!flagged)
                for (int jj = 0; jj < jn; jj += 4) {
                    // four codes per step, read as the uint32_t objects they are
                    const uint32_t cs[4] = {s_code[j0 + jj], s_code[j0 + jj + 1], s_code[j0 + jj + 2],
                                            s_code[j0 + jj + 3]};
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        nm |= ((cs[u] & lbits) == lbits && jj + u < jn) ? (1ull << (jj + u)) : 0ull;
                }
            while (__ballot(nm != 0)) {
                int j = 0;
                const bool has = nm != 0;
                if (has) {
                    j = j0 + __builtin_ctzll(nm);
                    nm &= nm - 1ull;
                }
                const uint64_t want = __ballot(has);
                if (has) s_q[nq + dev::lanes_below(want)] = ((uint32_t)lane << 7) | (uint32_t)j;
                nq += __popcll(want);
                if (nq >= 64) {
                    take(64);
                    __syncthreads();
                    if (s_fl[lane]) nm = 0;   // flagged meanwhile: nothing more to queue
                }
            }
        }
        if (nq > 0) take(nq);
        __syncthreads();
        flagged = s_fl[lane] != 0;
    };

    __shared__ int32_t s_seen[kDedup ? kSeen : 1];
    __shared__ int32_t s_list[kDedup ? kUniqCap : 1];
    __shared__ uint32_t s_bpre[kDedup ? 64 : 1], s_bs0[kDedup ? 64 : 1];
    bool done = __ballot(!flagged) == 0;
    for (int sb = 0; sb < BPW && !done; ++sb) {
        if (first + sb >= A.n) break;
        // block coordinates of sub-block sb (from its first lane)
        int sc[3];
        sc[0] = __shfl(bc[0], sb * CELLS, 64);
        sc[1] = __shfl(bc[1], sb * CELLS, 64);
        sc[2] = __shfl(bc[2], sb * CELLS, 64);
        float qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
        int ilo[3] = {0, 0, 0}, ihi[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) mc[a][i] = dev::uniform(dev::cell_centre(A.lo[a], 4 * sc[a] + i, A.dx[a]));
#pragma unroll
        for (int a = 0; a < D; ++a) {
            qlo[a] = (dev::cell_centre(A.lo[a], 4 * sc[a], A.dx[a]) - h) - A.eps[a];
            qhi[a] = (dev::cell_centre(A.lo[a], 4 * sc[a] + 3, A.dx[a]) + h) + A.eps[a];
            ilo[a] = dev::bin_of(qlo[a], A.bins.lo[a], A.bins.s[a], A.bins.B);
            ihi[a] = dev::bin_of(qhi[a], A.bins.lo[a], A.bins.s[a], A.bins.B);
        }
        // stage the faces whose box meets the query box (r: the lane's face record)
        auto stage = [&](bool has, int32_t f, const float *r) -> bool {
            bool keep = has;
#pragma unroll
            for (int a = 0; a < D; ++a) keep = keep && r[D * D + a] <= qhi[a] && r[D * D + D + a] >= qlo[a];
            const uint64_t mask = __ballot(keep);
            const int nk = __popcll(mask);
            if (nk == 0) return true;
            if (count + nk > kFlagCap) {
                test_staged(count);
                count = 0;
                done = __ballot(!flagged) == 0;
                if (done) return false;
            }
            if (keep) {
                const int pos = count + dev::lanes_below(mask);
#pragma unroll
                for (int k = 0; k < NF; ++k) s_f[k][pos] = r[k];
                s_code[pos] = face_code(sb, r + D * D);
            }
            count += nk;
            return true;
        };
        if constexpr (kDedup) {
            for_unique_candidates<D>(A.bins, A.faces.rec, ilo, ihi, s_seen, s_list, s_bpre, s_bs0, stage);
        } else {
            for_candidates(A.bins, ilo, ihi, [&](bool has, int32_t f, const int cur[3]) -> bool {
                // visit each face once: in the first bin of (its bins) x (query bins)
                float r[dev::kRecFloats<D>];
                bool first_bin = has;
                if (has) {
                    dev::load_rec<D>(A.faces.rec, f, r);
#pragma unroll
                    for (int a = 0; a < D; ++a)
                        first_bin = first_bin &&
                                    max(dev::bin_of(r[D * D + a], A.bins.lo[a], A.bins.s[a], A.bins.B), ilo[a]) == cur[a];
                }
                return stage(first_bin, f, (const float *)r);
            });
        }
    }
    if (!done && count > 0) test_staged(count);

    if (valid) A.cf[blk * CELLS + cell] = flagged ? 1 : 0;
    // block mark: OR over the block's cells
    const uint64_t fm = __ballot(valid && flagged);
    if (valid && cell == 0) {
        uint64_t bm = fm;
        if constexpr (CELLS < 64) bm = (fm >> (lane & ~(CELLS - 1))) & ((1ull << CELLS) - 1);
        A.pmark[blk] = bm ? 1 : 0;
    }
}

// Own-bin flag pass, the paper's face detection as printed (Sec. II-C-2 with
// Algorithm 1, bins of Sec. II-C-3): a cell looks only at the faces of the one
// bin that holds its centre (bin index function of the binning) and is
// flagged when its centre lies within Euclidean distance h of one of them
// (near_l2).  One wave: blocks first .. first + 64/4^D - 1 (one lane per
// cell).  The wave takes the distinct own bins of its lanes one after the
// other; each bin's faces are staged 64 at a time (one record per lane, in
// LDS) and the lanes of that bin test them, each stopping at its first near
// face.  Writes every cell flag and the block's pass mark (0 or 1).
template <int D>
__device__ __forceinline__ void flag_own_bin_wave(const FlagArgs<D> &A, int64_t first) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int RF = dev::kRecFloats<D>;
    __shared__ float s_v[64][D * D];
    const int lane = dev::lane_id();
    const int64_t blk = first + lane / CELLS;
    const bool valid = blk < A.n;
    const int cell = lane % CELLS;
    int bc[3] = {0, 0, 0};
    if (valid) dev::decode_key<D>(A.keys[blk], A.level, A.R[0], A.R[1], bc);
    float m[3] = {0.0f, 0.0f, 0.0f};
    m[0] = dev::cell_centre(A.lo[0], 4 * bc[0] + (cell & 3), A.dx[0]);
    m[1] = dev::cell_centre(A.lo[1], 4 * bc[1] + ((cell >> 2) & 3), A.dx[1]);
    if constexpr (D == 3) m[2] = dev::cell_centre(A.lo[2], 4 * bc[2] + (cell >> 4), A.dx[2]);
    int ib[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) ib[a] = dev::bin_of(m[a], A.bins.lo[a], A.bins.s[a], A.bins.B);
    const int mybin = (ib[2] * A.bins.B + ib[1]) * A.bins.B + ib[0];   // B^D < 2^31 (checked when binning)
    bool flagged = false;
    bool done = !valid;
    while (true) {
        const uint64_t open = __ballot(!done);
        if (!open) break;
        const int leader = __builtin_ctzll(open);
        const int bin = __builtin_amdgcn_readlane(mybin, leader);
        const bool mine = !done && mybin == bin;
        const uint32_t s0 = A.bins.off[bin], s1 = A.bins.off[bin + 1];
        for (uint32_t c0 = s0; c0 < s1; c0 += dev::kWave) {
            if (!__ballot(mine && !flagged)) break;   // every cell of this bin decided
            const uint32_t e = c0 + (uint32_t)lane;
            if (e < s1) {
                const int32_t f = A.bins.ids[e];
                float r[RF];
                if (f >= 0 && (int64_t)f < A.bins.F) {
                    dev::load_rec<D>(A.faces.rec, f, r);
                } else {
#pragma unroll
                    for (int k = 0; k < RF; ++k) r[k] = __builtin_nanf("");   // never near
                }
#pragma unroll
                for (int k = 0; k < D * D; ++k) s_v[lane][k] = r[k];
            }
            dev::wave_sync();
            const int nf = (int)min(s1 - c0, (uint32_t)dev::kWave);
            if (mine && !flagged)
                for (int j = 0; j < nf; ++j) {
                    float v[D * D];
#pragma unroll
                    for (int k = 0; k < D * D; ++k) v[k] = s_v[j][k];
                    if (dev::near_l2<D>(v, m, A.h)) {
                        flagged = true;
                        break;
                    }
                }
            dev::wave_sync();
        }
        done = done || mine;
    }
    if (valid) A.cf[blk * CELLS + cell] = flagged ? 1 : 0;
    const uint64_t fm = __ballot(valid && flagged);
    if (valid && cell == 0) {
        uint64_t bm = fm;
        if constexpr (CELLS < 64) bm = (fm >> (lane & ~(CELLS - 1))) & ((1ull << CELLS) - 1);
        A.pmark[blk] = bm ? 1 : 0;
    }
}

// Mark propagation of the own-bin pass (Sec. II-C-3), one step in two
// launches so that a step grows the marked set by exactly one ring whatever
// the order of the threads: (1) every unmarked level-l neighbour (faces,
// edges, corners; inside the domain; present at level l) of a block whose
// pass mark is 1 (flagged) or 3 (propagated) gets the intermediate value 4;
// (2) every 4 becomes 3.  One thread per (block, neighbour position).
template <int D>
__device__ __forceinline__ void prop_spread_item(const uint32_t *keys, int64_t n, uint8_t *pm, int l, int R0, int R1,
                                                 int R2, int64_t t) {
    constexpr int NNB = D == 3 ? 26 : 8;
    const int64_t i = t / NNB;
    const uint8_t p = pm[i];
    if (p != 1 && p != 3) return;
    int k = (int)(t % NNB);
    k += k >= NNB / 2 ? 1 : 0;   // skip the centre of the 3^D stencil
    const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = D == 3 ? k / 9 - 1 : 0;
    int c[3];
    dev::decode_key<D>(keys[i], l, R0, R1, c);
    const int ext[3] = {R0 << l, R1 << l, R2 << l};
    int nc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
    if (nc[0] < 0 || nc[0] >= ext[0] || nc[1] < 0 || nc[1] >= ext[1]) return;
    if (D == 3 && (nc[2] < 0 || nc[2] >= ext[2])) return;
    const uint32_t kn = dev::encode_key<D>(nc, l, R0, R1);
    const int64_t j = dev::lower_bound_u32(keys, n, kn);
    if (j < n && keys[j] == kn && pm[j] == 0) pm[j] = 4;
}

// Face-centric flag pass.  A cell's flag is an OR over faces of one FP32 test
// (sat_triangle / sat_segment at the cell centre, half-width h), so it can be
// gathered from the faces' side as well: each face visits the cells whose
// centre lies within h + eps of its box on every axis (a superset of the cells
// whose box-axis tests it passes) and sets the flag of each cell it is not
// separated from.  The work is a few cells per face, spread over every lane of
// the chip, where the cell-centric pass is as long as its busiest block's wave
// (a coarse block's query box spans hundreds of bins).  Cells of blocks that
// do not exist at the level are skipped: a dense table over the level's block
// grid holds each block's index; an entry counts only when it is below n and
// the level's key at that index is the key of the grid position, so the table
// is never cleared and stale entries read as absent.  At level 0 every block
// exists and the index is the linear one.  Cell flags and block marks must
// start at zero; only ones are stored, so faces that meet the same cell race
// harmlessly.
// Faces per wave G (4, 8 or 16) is picked per launch: small face counts take
// small G so that the pass still has several waves per SIMD to hide the table
// and flag reads (measured on MI355X: 20,480 faces 68 -> 54 us with G = 4;
// 327,680 faces 295 us with G = 16, 438 us with G = 4).
constexpr int kFaceFlagWaves = 4;   // waves per workgroup
constexpr int kFaceFlagInts = 10;   // per-face words of the wave's face table
inline int face_flag_g(int64_t faces, int n_cu) {
    const int64_t want = 8 * 4 * (int64_t)n_cu;   // waves: eight per SIMD
    return faces >= 16 * want ? 16 : (faces >= 8 * want ? 8 : 4);
}

template <int D>
struct FaceFlagArgs {
    const float *rec;         // F x kRecFloats<D>
    int64_t F;
    int NB[3];                // blocks per axis at this level (roots << level)
    const uint32_t *table;    // NB0 NB1 NB2 entries, x fastest; null at level 0
    const uint32_t *keys;     // the level's keys (n), to validate table entries
    int64_t n;
    int level;
    int R[2];                 // roots along x and y (key encoding)
    float lo[3];
    float dx[3];              // cell size at this level
    float eps[3];
    float h;
    uint8_t *cf;              // n x 4^D, zeroed
    uint8_t *pmark;           // n, zeroed
};

// One wave: faces face0 .. face0 + G - 1.  The (face, cell) pairs of
// its faces are listed in face order and taken 64 at a time, one per lane.  A
// face with a non-finite coordinate has no pairs (its input is rejected
// anyway; the batched form reports it after the run).  Pair counts are 64-bit:
// a face much larger than the level's cells can have more than 2^32 / 16
// pairs; index arithmetic stays 32-bit while the wave's total fits.
template <int D, int G>
__device__ __forceinline__ void flag_faces_wave(const FaceFlagArgs<D> &A, int64_t face0,
                                                float (*s_rec)[dev::kRecFloats<D>], int (*s_i)[kFaceFlagInts]) {
    constexpr int RF = dev::kRecFloats<D>;
    constexpr int CELLS = D == 3 ? 64 : 16;
    static_assert(G >= 2 && G <= 64 && (G & (G - 1)) == 0, "face search takes log2(G) steps");
    const int lane = dev::lane_id();
    uint64_t cnt = 0;
    if (lane < G) {
        const int64_t f = face0 + lane;
        int ilo[3] = {0, 0, 0}, n[3] = {0, 1, 1};
        if (f < A.F) {
            float r[RF];
            dev::load_rec<D>(A.rec, f, r);
#pragma unroll
            for (int k = 0; k < RF; ++k) s_rec[lane][k] = r[k];
            bool finite = true;
#pragma unroll
            for (int k = 0; k < D * D + 2 * D; ++k) finite = finite && isfinite(r[k]);
            cnt = finite ? 1u : 0u;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                // cells i with centre lo + (i + 1/2) dx in [min - h - eps, max + h + eps]
                const int nc = 4 * A.NB[a];
                const double lo = A.lo[a], dx = A.dx[a], reach = (double)A.h + (double)A.eps[a];
                const double xl = fmin(fmax(((double)r[D * D + a] - reach - lo) / dx - 0.5, -1.0), (double)nc);
                const double xh = fmax(fmin(((double)r[D * D + D + a] + reach - lo) / dx - 0.5, (double)nc), -1.0);
                const int i0 = max(0, (int)ceil(xl));
                const int i1 = min(nc - 1, (int)floor(xh));
                ilo[a] = i0;
                n[a] = finite ? max(0, i1 - i0 + 1) : 0;
                cnt *= (uint64_t)n[a];
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            s_i[lane][a] = ilo[a];
            s_i[lane][3 + a] = n[a];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
            s_i[lane][8 + a] = n[a] > 1 ? (int)(uint32_t)((0x100000000ull + (uint64_t)n[a] - 1u) / (uint64_t)n[a]) : 0;
    }
    // pair indices below 2^16 (every face of the wave): quotients by the
    // per-axis cell counts as multiply-high by ceil(2^32 / n), exact there
    const bool small = __ballot(cnt > 65536u) == 0ull;
    // 64-bit inclusive wave prefix of the pair counts
    uint64_t incl = cnt;
#pragma unroll
    for (int d = 1; d < dev::kWave; d <<= 1) {
        const uint64_t y = __shfl_up(incl, d, dev::kWave);
        if (lane >= d) incl += y;
    }
    const uint64_t total = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(incl >> 32), dev::kWave - 1) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)incl, dev::kWave - 1);
    if (lane < G) {
        const uint64_t pre = incl - cnt;
        s_i[lane][6] = (int)(uint32_t)pre;
        s_i[lane][7] = (int)(uint32_t)(pre >> 32);
    }
    dev::wave_sync();
    // A pair that needs the separating-axis test (its block exists at the
    // level, its cell is not flagged yet) is queued with its cell centre,
    // block and face; the queue is tested 64 pairs at a time, one per lane, so
    // that the lanes of a step whose pairs were dropped do not idle through the
    // test.  The test and what it writes are those of the pair itself.
    constexpr int QCAP = 128;   // below 64 between steps, at most 64 added per step
    __shared__ float s_qm[kFaceFlagWaves][3][QCAP];
    __shared__ uint32_t s_qb[kFaceFlagWaves][QCAP];
    __shared__ uint32_t s_qk[kFaceFlagWaves][QCAP];
    const int wq = (int)(threadIdx.x / dev::kWave);
    int nq = 0;   // wave-uniform
    auto test = [&](int take) {
        dev::wave_sync();
        float m[3] = {0.0f, 0.0f, 0.0f};
        uint32_t blk = 0, kc = 0;
        if (lane < take) {
#pragma unroll
            for (int a = 0; a < 3; ++a) m[a] = s_qm[wq][a][lane];
            blk = s_qb[wq][lane];
            kc = s_qk[wq][lane];
        }
        dev::wave_sync();
        if (lane < nq - take) {
#pragma unroll
            for (int a = 0; a < 3; ++a) s_qm[wq][a][lane] = s_qm[wq][a][take + lane];
            s_qb[wq][lane] = s_qb[wq][take + lane];
            s_qk[wq][lane] = s_qk[wq][take + lane];
        }
        nq -= take;
        if (lane < take) {
            const int k = (int)(kc >> 8), cell = (int)(kc & 255u);
            float vv[D * D];
#pragma unroll
            for (int j = 0; j < D * D; ++j) vv[j] = s_rec[k][j];
            bool hit;
            if constexpr (D == 3) hit = dev::sat_triangle(vv, m, A.h);
            else hit = dev::sat_segment(vv, m, A.h);
            if (hit) {
                A.cf[(int64_t)blk * CELLS + cell] = 1;
                A.pmark[blk] = 1;
            }
        }
    };
    // pair v: its cell, then whether it is queued
    auto pair = [&](auto v, float (&m)[3], uint32_t &qblk, uint32_t &qkc) -> bool {
        using T = decltype(v);
        auto pre_of = [&](int k) -> T {
            return (T)(((uint64_t)(uint32_t)s_i[k][7] << 32) | (uint32_t)s_i[k][6]);
        };
        int k = 0;   // the last face whose pairs start at or before v
#pragma unroll
        for (int step = G / 2; step >= 1; step >>= 1)
            if (pre_of(k + step) <= v) k += step;
        const T u = v - pre_of(k);
        int g[3] = {0, 0, 0};
        const T n0 = (T)s_i[k][3], n1 = (T)s_i[k][4];
        T q0, q1;
        if (sizeof(T) == 4 && small) {
            q0 = n0 > 1 ? (T)__umulhi((uint32_t)u, (uint32_t)s_i[k][8]) : u;
            q1 = n1 > 1 ? (T)__umulhi((uint32_t)q0, (uint32_t)s_i[k][9]) : q0;
        } else {
            q0 = u / n0;
            q1 = q0 / n1;
        }
        g[0] = s_i[k][0] + (int)(u - q0 * n0);
        if constexpr (D == 3) {
            g[1] = s_i[k][1] + (int)(q0 - q1 * n1);
            g[2] = s_i[k][2] + (int)q1;
        } else {
            g[1] = s_i[k][1] + (int)q0;
        }
#pragma unroll
        for (int a = 0; a < D; ++a) m[a] = dev::cell_centre(A.lo[a], g[a], A.dx[a]);
        int64_t blk = (int64_t)(g[1] >> 2) * A.NB[0] + (g[0] >> 2);
        int cell = (g[0] & 3) | ((g[1] & 3) << 2);
        if constexpr (D == 3) {
            blk += (int64_t)(g[2] >> 2) * A.NB[0] * A.NB[1];
            cell |= (g[2] & 3) << 4;
        }
        if (A.table) {
            const uint32_t t = A.table[blk];
            const int bc[3] = {g[0] >> 2, g[1] >> 2, D == 3 ? g[2] >> 2 : 0};
            if ((int64_t)t >= A.n || A.keys[t] != dev::encode_key<D>(bc, A.level, A.R[0], A.R[1]))
                return false;   // no such block at this level
            blk = t;
        }
        if (A.cf[blk * CELLS + cell]) return false;   // flagged already
        qblk = (uint32_t)blk;   // a block index of the level (below 2^32)
        qkc = ((uint32_t)k << 8) | (uint32_t)cell;
        return true;
    };
    auto step = [&](bool valid, auto v) {
        float m[3] = {0.0f, 0.0f, 0.0f};
        uint32_t qblk = 0, qkc = 0;
        const bool want = valid && pair(v, m, qblk, qkc);
        const uint64_t bm = __ballot(want);
        if (want) {
            const int at = nq + dev::lanes_below(bm);
#pragma unroll
            for (int a = 0; a < 3; ++a) s_qm[wq][a][at] = m[a];
            s_qb[wq][at] = qblk;
            s_qk[wq][at] = qkc;
        }
        nq += __popcll(bm);
        if (nq >= dev::kWave) test(dev::kWave);
    };
    if (total <= 0xFFFFFFFFull) {
        const uint32_t tot = (uint32_t)total;
        for (uint32_t c0 = 0; c0 < tot; c0 += dev::kWave) step(c0 + lane < tot, (uint32_t)(c0 + lane));
    } else {
        for (uint64_t c0 = 0; c0 < total; c0 += dev::kWave) step(c0 + lane < total, (uint64_t)(c0 + lane));
    }
    if (nq > 0) test(nq);
}

// 2:1 balance: a block of level m marked in this pass needs every neighbour
// position (faces, edges, corners) inside the domain to exist at level m;
// where it does not, the covering level-(m-1) leaf is marked.  One thread per
// (block, neighbour position).  Blocks are created as whole sibling groups,
// the children of a refined parent, so a level-m position exists exactly when
// its level-(m-1) parent exists and is not a leaf: a neighbour with the
// block's own parent exists, and any other takes one binary search, for its
// parent in level m-1 (refined: it exists; a leaf: marked; missing: the 2:1
// rule was broken below, an error).
template <int D>
__device__ __forceinline__ void ripple_item(const uint32_t *keys_m, int64_t n_m, const uint8_t *pm_m, int m,
                                            const uint32_t *keys_p, int64_t n_p, const uint8_t *leaf_p, uint8_t *pm_p,
                                            int R0, int R1, int R2, uint32_t *err, int64_t t) {
    constexpr int NNB = D == 3 ? 26 : 8;
    {
        const int64_t i = t / NNB;
        if (!pm_m[i]) return;
        int k = (int)(t % NNB);
        k += k >= NNB / 2 ? 1 : 0;   // skip the centre of the 3^D stencil
        const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = D == 3 ? k / 9 - 1 : 0;
        int c[3];
        dev::decode_key<D>(keys_m[i], m, R0, R1, c);
        const int ext[3] = {R0 << m, R1 << m, R2 << m};
        int nc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
        if (nc[0] < 0 || nc[0] >= ext[0] || nc[1] < 0 || nc[1] >= ext[1]) return;
        if (D == 3 && (nc[2] < 0 || nc[2] >= ext[2])) return;
        int pc[3] = {nc[0] >> 1, nc[1] >> 1, D == 3 ? nc[2] >> 1 : 0};
        if (pc[0] == c[0] >> 1 && pc[1] == c[1] >> 1 && (D == 2 || pc[2] == c[2] >> 1)) return;   // a sibling
        const uint32_t kp = dev::encode_key<D>(pc, m - 1, R0, R1);
        const int64_t jp = dev::lower_bound_u32(keys_p, n_p, kp);
        if (jp < n_p && keys_p[jp] == kp) {
            if (leaf_p[jp]) pm_p[jp] = 2;
        } else {
            atomicOr(err, 1u);
        }
    }
}

// Marked blocks of level m: become parents (leaf 0, export mark = pass mark)
// and their keys are compacted in order into mk.
__device__ __forceinline__ void mark_parents_item(const uint32_t *keys, const uint8_t *pm, const uint32_t *pos,
                                                  uint8_t *leaf, uint8_t *mark, uint32_t *mk, int64_t i) {
    {
        const uint8_t p = pm[i];
        if (!p) return;
        leaf[i] = 0;
        mark[i] = p;
        mk[pos[i]] = keys[i];
    }
}

// Existing blocks of level m+1 move to their place in the merged list.
template <int CELLS>
__device__ __forceinline__ void merge_old_item(const uint32_t *keys, const uint8_t *leaf, const uint8_t *mark,
                                               const uint8_t *cf, const uint32_t *mk, int64_t n_mk, int D,
                                               uint32_t *nkeys, uint8_t *nleaf, uint8_t *nmark, uint8_t *ncf,
                                               int64_t i, int64_t cap = INT64_MAX) {
    {
        const uint32_t k = keys[i];
        const int64_t r = dev::lower_bound_u32(mk, n_mk, k >> D);
        const int64_t p = i + (r << D);
        if (p >= cap) return;   // batched plans: out of planned capacity (reported by the count step)
        nkeys[p] = k;
        nleaf[p] = leaf[i];
        nmark[p] = mark[i];
        if (ncf) {   // one 16- or 64-byte row: 16-byte moves
#pragma unroll
            for (int c = 0; c < CELLS / 16; ++c) {
                uint4 x;
                __builtin_memcpy(&x, cf + i * CELLS + 16 * c, 16);
                __builtin_memcpy(ncf + p * CELLS + 16 * c, &x, 16);
            }
        }
    }
}

// Children of the marked parents, placed after the existing keys below them.
template <int CELLS>
__device__ __forceinline__ void children_item(const uint32_t *mk, const uint32_t *keys_old, int64_t n_old, int D,
                                              uint32_t *nkeys, uint8_t *nleaf, uint8_t *nmark, uint8_t *ncf,
                                              int64_t t, int64_t cap = INT64_MAX) {
    {
        const int64_t pi = t >> D;
        const uint32_t ci = (uint32_t)(t & ((1 << D) - 1));
        const uint32_t parent = mk[pi];
        const int64_t below = dev::lower_bound_u32(keys_old, n_old, parent << D);
        const int64_t p = below + t;
        if (p >= cap) return;
        nkeys[p] = (parent << D) | ci;
        nleaf[p] = 1;
        nmark[p] = 0;
        if (ncf) {
            const uint4 z = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
            for (int c = 0; c < CELLS / 16; ++c) __builtin_memcpy(ncf + p * CELLS + 16 * c, &z, 16);
        }
    }
}



// ===========================================================================
// Link fractions and their adjoint (paper Sec. II-C-1)
// ===========================================================================
constexpr int kLinkCap = 32;   // staged faces per wave (LDS per wave bounds occupancy)

template <int D, int Q>
struct LinkArgs {
    dev::Faces faces;
    dev::BinGrid bins;
    const uint32_t *keys;
    int64_t n;
    int level;
    int R[3];
    float lo[3];
    float dx[3];
    float eps[3];
    // Candidate faces per block (list mode): the faces of block b are
    // list[loff[b] .. loff[b + 1]).  Null: the wave walks the bins under the
    // block instead.
    const uint32_t *loff;
    const int32_t *list;
    uint32_t list_cap;     // entries allocated for the lists (reads stay below it)
    uint64_t *node_key;    // node rows (staging rows in walk mode)
    float *q;
    int32_t *face;
};

// Candidate faces staged in LDS by one link wave: vertices (3D: and the FP32
// normal n = (b - a) x (c - a), |E1|_1, |E2|_1 and S = sum |n_a dx_a|), the
// face id and the face's near code (one bit per (axis, cell position) of the
// block it was staged for).
// With kNorms (3D) the face's L1 norms |E1|_1, |E2|_1 and sum_a |n_a dx_a|
// are staged too (f[12..14]); without them the filter forms them again from
// the staged corners and normal, with the same expressions, so the results are
// the same and the staging area is a fifth smaller.
template <int D, int CAP = kLinkCap, bool kNorms = true>
struct LinkStaged {
    static constexpr int NF = D == 3 ? (kNorms ? 15 : 12) : 4;
    float f[NF][CAP];
    int32_t id[CAP];
    uint32_t code[CAP];
};

template <int D, int CAP, bool kN>
__device__ __forceinline__ void link_stage(LinkStaged<D, CAP, kN> &S, int pos, int32_t f, const float *r, const float dx[3],
                                           uint32_t code) {
    S.id[pos] = f;
    if constexpr (D == 3) {
        const float *v = r;
        const float e10 = v[3] - v[0], e11 = v[4] - v[1], e12 = v[5] - v[2];
        const float e20 = v[6] - v[0], e21 = v[7] - v[1], e22 = v[8] - v[2];
#pragma unroll
        for (int k = 0; k < 9; ++k) S.f[k][pos] = v[k];
        const float n0 = e11 * e22 - e12 * e21;
        const float n1 = e12 * e20 - e10 * e22;
        const float n2 = e10 * e21 - e11 * e20;
        S.f[9][pos] = n0;
        S.f[10][pos] = n1;
        S.f[11][pos] = n2;
        if constexpr (kN) {
            S.f[12][pos] = fabsf(e10) + fabsf(e11) + fabsf(e12);
            S.f[13][pos] = fabsf(e20) + fabsf(e21) + fabsf(e22);
            S.f[14][pos] = fabsf(n0 * dx[0]) + fabsf(n1 * dx[1]) + fabsf(n2 * dx[2]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) S.f[k][pos] = r[k];
    }
    S.code[pos] = code;
}

// FP32 filter of staged face j for a link origin o over all direction pairs.
// With T = o - a, E1 = b - a, E2 = c - a the solution of o + t D = a + u E1 +
// v E2 is det = D.n, u = D.(T x E2)/det, v = D.(E1 x T)/det, t = -(T.n)/det;
// T x E2, E1 x T and T.n do not depend on D, and D = c_i dx has entries in
// {-dx, 0, dx}, so a direction costs a few additions, and the opposite
// direction has the same u, v and t of the opposite sign; NP direction pairs
// (directions 1 + 2p, p < NP).  Each quantity carries an absolute rounding
// error bounded by 2^-21 times the product of the L1 norms of its factors
// (the direction counted as its largest cell size); margins of 2^-20 times
// those products are applied.  Returns the pairs that may meet the face (every true hit passes:
// |t| <= 1 on the face's plane and, unless D.n is too small to have a known
// sign, barycentrics inside).  With kSure, *sure tells whether some pair
// certainly meets it (the same tests narrowed by the margins: the exact u, v,
// 1 - u - v and 1 - |t| are then positive by at least half a margin, so the
// FP64 decision finds a hit for one of the pair's two directions).
template <int D, int NP, bool kSure, int CAP, bool kN>
__device__ __forceinline__ uint32_t link_filter(const LinkStaged<D, CAP, kN> &S, int j, const float o[3], const float dx[3],
                                                bool *sure) {
    // The pair-independent sums of margins are formed once: comparing
    // atn - (MD + MT) <= ad instead of atn <= (ad + MD) + MT (and so on) moves
    // each bound by a rounding of at most a sixteenth of a margin, within the
    // half margin the error bounds leave free.
    uint32_t cm = 0;
    bool cs = false;
    if constexpr (D == 3) {
        const float T0 = o[0] - S.f[0][j], T1 = o[1] - S.f[1][j], T2 = o[2] - S.f[2][j];
        const float e10 = S.f[3][j] - S.f[0][j], e11 = S.f[4][j] - S.f[1][j], e12 = S.f[5][j] - S.f[2][j];
        const float e20 = S.f[6][j] - S.f[0][j], e21 = S.f[7][j] - S.f[1][j], e22 = S.f[8][j] - S.f[2][j];
        const float n0 = S.f[9][j], n1 = S.f[10][j], n2 = S.f[11][j];
        float n1n, n2n;
        if constexpr (kN) {
            n1n = S.f[12][j];
            n2n = S.f[13][j];
        } else {
            n1n = fabsf(e10) + fabsf(e11) + fabsf(e12);
            n2n = fabsf(e20) + fabsf(e21) + fabsf(e22);
        }
        const float nT = fabsf(T0) + fabsf(T1) + fabsf(T2);
        const float mx_ = fmaxf(fmaxf(dx[0], dx[1]), dx[2]) * 9.5367431640625e-07f;  // dx * 2^-20
        const float MU = mx_ * nT * n2n;
        const float MV = mx_ * n1n * nT;
        const float MD = mx_ * n1n * n2n;
        const float MT = 9.5367431640625e-07f * nT * n1n * n2n;
        const float p10 = (T1 * e22 - T2 * e21) * dx[0];
        const float p11 = (T2 * e20 - T0 * e22) * dx[1];
        const float p12 = (T0 * e21 - T1 * e20) * dx[2];
        const float p20 = (e11 * T2 - e12 * T1) * dx[0];
        const float p21 = (e12 * T0 - e10 * T2) * dx[1];
        const float p22 = (e10 * T1 - e11 * T0) * dx[2];
        const float d0 = n0 * dx[0], d1 = n1 * dx[1], d2 = n2 * dx[2];
        const float atn = fabsf((T0 * n0 + T1 * n1) + T2 * n2);
        const float MDT = MD + MT, MUVD = (MU + MV) + MD;
        const float t_lo = atn - MDT;   // |t| <= 1 possible: t_lo <= |D.n|
        const float t_hi = atn + MDT;   // |t| < 1 certain: t_hi <= |D.n|
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int i = 1 + 2 * p;
            const int c0 = dir_c<D>(i, 0), c1 = dir_c<D>(i, 1), c2 = dir_c<D>(i, 2);
            // signed sums over the direction's non-zero components, started at the first of them (an
            // addition to 0.0f would stay in the code: it only changes the sign of a zero, which no
            // comparison below sees)
            float den = 0.0f, nu = 0.0f, nv = 0.0f;
            bool started = false;
            auto term = [&](int c, float d, float pu, float pv) {
                if (!c) return;
                const float sd = c > 0 ? d : -d, su_ = c > 0 ? pu : -pu, sv_ = c > 0 ? pv : -pv;
                if (started) {
                    den += sd;
                    nu += su_;
                    nv += sv_;
                } else {
                    den = sd;
                    nu = su_;
                    nv = sv_;
                    started = true;
                }
            };
            term(c0, d0, p10, p20);
            term(c1, d1, p11, p21);
            term(c2, d2, p12, p22);
            const float ad = fabsf(den);
            const bool neg = den < 0.0f;
            const float su = neg ? -nu : nu;
            const float sv = neg ? -nv : nv;
            const float suv = su + sv;
            const bool bary = (su >= -MU) & (sv >= -MV) & (suv - ad <= MUVD);
            cm |= ((t_lo <= ad) & ((ad <= MD) | bary)) ? (1u << p) : 0u;
            if constexpr (kSure)
                cs = cs | ((ad > MD) & (t_hi <= ad) & (su >= MU) & (sv >= MV) & (suv + MUVD <= ad));
        }
    } else {
        const float w0 = S.f[0][j] - o[0], w1 = S.f[1][j] - o[1];
        const float e0 = S.f[2][j] - S.f[0][j], e1 = S.f[3][j] - S.f[1][j];
        const float nw = fabsf(w0) + fabsf(w1), ne = fabsf(e0) + fabsf(e1);
        const float mx_ = fmaxf(dx[0], dx[1]) * 9.5367431640625e-07f;
        const float MD = mx_ * ne, MS = mx_ * nw, MW = 9.5367431640625e-07f * nw * ne;
        const float awxe = fabsf(w0 * e1 - w1 * e0);
        const float MDW = MD + MW, MSD = MS + MD;
        const float t_lo = awxe - MDW, t_hi = awxe + MDW;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int i = 1 + 2 * p;
            const float D0 = (float)dir_c<D>(i, 0) * dx[0], D1 = (float)dir_c<D>(i, 1) * dx[1];
            const float den = D0 * e1 - D1 * e0;
            const float ad = fabsf(den);
            const float sn = w0 * D1 - w1 * D0;
            const float ss = den < 0.0f ? -sn : sn;
            const bool seg = (ss >= -MS) & (ss - ad <= MSD);
            cm |= ((t_lo <= ad) & ((ad <= MD) | seg)) ? (1u << p) : 0u;
            if constexpr (kSure) cs = cs | ((ad > MD) & (t_hi <= ad) & (ss >= MS) & (ss + MSD <= ad));
        }
    }
    if constexpr (kSure) *sure = cs;
    return cm;
}

// Whether any direction pair can pass the filter for staged face j and origin
// o: the filter's |t| test with the largest |D . n| of any direction,
// S = sum |n_a dx_a| (3D; always in 2D).
template <int D, int CAP, bool kN>
__device__ __forceinline__ bool link_reach(const LinkStaged<D, CAP, kN> &S, int j, const float o[3], const float dx[3]) {
    if constexpr (D == 3) {
        const float T0 = o[0] - S.f[0][j], T1 = o[1] - S.f[1][j], T2 = o[2] - S.f[2][j];
        const float n0 = S.f[9][j], n1 = S.f[10][j], n2 = S.f[11][j];
        float n1n, n2n, Sn;
        if constexpr (kN) {
            n1n = S.f[12][j];
            n2n = S.f[13][j];
            Sn = S.f[14][j];
        } else {
            n1n = (fabsf(S.f[3][j] - S.f[0][j]) + fabsf(S.f[4][j] - S.f[1][j])) + fabsf(S.f[5][j] - S.f[2][j]);
            n2n = (fabsf(S.f[6][j] - S.f[0][j]) + fabsf(S.f[7][j] - S.f[1][j])) + fabsf(S.f[8][j] - S.f[2][j]);
            Sn = (fabsf(n0 * dx[0]) + fabsf(n1 * dx[1])) + fabsf(n2 * dx[2]);
        }
        const float nT = fabsf(T0) + fabsf(T1) + fabsf(T2);
        const float mx_ = fmaxf(fmaxf(dx[0], dx[1]), dx[2]) * 9.5367431640625e-07f;
        const float MD = mx_ * n1n * n2n;
        const float MT = 9.5367431640625e-07f * nT * n1n * n2n;
        return fabsf((T0 * n0 + T1 * n1) + T2 * n2) <= Sn + MD + MT;
    } else {
        return true;
    }
}

// FP64 decision for staged face j, direction Dv (the first direction of a
// pair) and origin o: the segment-triangle test (Moller-Trumbore, two-sided,
// closed) in the same expression order as the definition; returns t of Dv,
// or NaN when the line misses the face or det = 0.  The opposite direction
// hits at -t (negating D negates P, det and t exactly), so the pair has a
// link in direction Dv when t is in [0, 1] and in -Dv when -t is.
template <int D, int CAP, bool kN>
__device__ __forceinline__ double link_decide(const LinkStaged<D, CAP, kN> &S, int j, const double o[3], const float dir[3]) {
    const double nan = __builtin_nan("");
    if constexpr (D == 3) {
        const double a0 = S.f[0][j], a1 = S.f[1][j], a2 = S.f[2][j];
        const double E1[3] = {(double)S.f[3][j] - a0, (double)S.f[4][j] - a1, (double)S.f[5][j] - a2};
        const double E2[3] = {(double)S.f[6][j] - a0, (double)S.f[7][j] - a1, (double)S.f[8][j] - a2};
        const double T[3] = {o[0] - a0, o[1] - a1, o[2] - a2};
        const double Dv[3] = {(double)dir[0], (double)dir[1], (double)dir[2]};
        const double P[3] = {Dv[1] * E2[2] - Dv[2] * E2[1], Dv[2] * E2[0] - Dv[0] * E2[2],
                             Dv[0] * E2[1] - Dv[1] * E2[0]};
        const double det = E1[0] * P[0] + E1[1] * P[1] + E1[2] * P[2];
        if (det == 0.0) return nan;
        const double u = (T[0] * P[0] + T[1] * P[1] + T[2] * P[2]) / det;
        if (u < 0.0 || u > 1.0) return nan;
        const double Qv[3] = {T[1] * E1[2] - T[2] * E1[1], T[2] * E1[0] - T[0] * E1[2], T[0] * E1[1] - T[1] * E1[0]};
        const double v = (Dv[0] * Qv[0] + Dv[1] * Qv[1] + Dv[2] * Qv[2]) / det;
        if (v < 0.0 || u + v > 1.0) return nan;
        return (E2[0] * Qv[0] + E2[1] * Qv[1] + E2[2] * Qv[2]) / det;
    } else {
        const double a0 = S.f[0][j], a1 = S.f[1][j];
        const double e0 = (double)S.f[2][j] - a0, e1 = (double)S.f[3][j] - a1;
        const double D0 = (double)dir[0], D1 = (double)dir[1];
        const double den = D0 * e1 - D1 * e0;
        if (den == 0.0) return nan;
        const double w0 = a0 - o[0], w1 = a1 - o[1];
        const double t = (w0 * e1 - w1 * e0) / den;
        const double sp = (w0 * D1 - w1 * D0) / den;
        if (!(sp >= 0.0 && sp <= 1.0)) return nan;
        return t;
    }
}

// Link box of sub-block sb of a wave (block coordinates sc): per axis the
// bounds of each cell position's link box (cell +- one cell, widened by eps;
// wave-uniform, kept in scalar registers), the block's link box [qlo, qhi]
// and the bins under it.
template <int D>
struct LinkBox {
    float mlo[D][4], mhi[D][4];
    float qlo[3], qhi[3];
    int ilo[3], ihi[3];
};

template <int D, int Q>
__device__ __forceinline__ void link_box(const LinkArgs<D, Q> &A, const int sc[3], LinkBox<D> &bx) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bx.qlo[a] = bx.qhi[a] = 0.0f;
        bx.ilo[a] = bx.ihi[a] = 0;
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float c = dev::cell_centre(A.lo[a], 4 * sc[a] + i, A.dx[a]);
            bx.mlo[a][i] = dev::uniform((c - A.dx[a]) - A.eps[a]);
            bx.mhi[a][i] = dev::uniform((c + A.dx[a]) + A.eps[a]);
        }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        bx.qlo[a] = (dev::cell_centre(A.lo[a], 4 * sc[a], A.dx[a]) - A.dx[a]) - A.eps[a];
        bx.qhi[a] = (dev::cell_centre(A.lo[a], 4 * sc[a] + 3, A.dx[a]) + A.dx[a]) + A.eps[a];
        bx.ilo[a] = dev::bin_of(bx.qlo[a], A.bins.lo[a], A.bins.s[a], A.bins.B);
        bx.ihi[a] = dev::bin_of(bx.qhi[a], A.bins.lo[a], A.bins.s[a], A.bins.B);
    }
}

// Offers the candidate faces of block blk (sub-block sb of the wave, link box
// bx) to the staging area: the faces whose bounding box meets the block's link
// box, from the block's candidate list (list mode) or from the bins under the
// box (each face once, in the first bin of (its bins) x (the box's bins)).  A
// round of 64 candidates can keep more faces than the area holds: they are
// staged in pieces that fit, flush(count) testing and emptying the area
// between pieces (whole wave).  Returns the number of faces left staged.
template <int D, int Q, class Flush>
__device__ __forceinline__ int link_gather(const LinkArgs<D, Q> &A, int64_t blk, int sb, const LinkBox<D> &bx,
                                           LinkStaged<D> &S, int count, Flush &&flush) {
    const int lane = dev::lane_id();
    auto face_code = [&](const float *bb) -> uint32_t {   // bb: min[D], max[D]
        uint32_t c = 0;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                c |= (bb[a] <= bx.mhi[a][i] && bb[D + a] >= bx.mlo[a][i]) ? (1u << (4 * a + i)) : 0u;
        return c << (sb * 4 * D);
    };
    auto round = [&](bool has, int32_t f, const int *cur) {
        bool keep = false;
        float r[dev::kRecFloats<D>];
        const float *bb = r + D * D;   // min then max
        if (has) {
            dev::load_rec<D>(A.faces.rec, f, r);
            keep = true;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (cur) {
                    const int fb = max(dev::bin_of(bb[a], A.bins.lo[a], A.bins.s[a], A.bins.B), bx.ilo[a]);
                    keep = keep && fb == cur[a];
                }
                keep = keep && bb[a] <= bx.qhi[a] && bb[D + a] >= bx.qlo[a];
            }
        }
        uint64_t rest = __ballot(keep);
        while (rest) {
            if (count > 0 && count + __popcll(rest) > kLinkCap) {
                flush(count);
                count = 0;
            }
            const bool now = ((rest >> lane) & 1ull) && dev::lanes_below(rest) < kLinkCap - count;
            const uint64_t part = __ballot(now);
            rest &= ~part;
            const int pos = count + dev::lanes_below(part);
            count += __popcll(part);
            if (now) link_stage<D>(S, pos, f, r, A.dx, face_code(bb));
        }
    };
    if (A.list) {
        const uint32_t s0 = A.loff[blk], s1 = min(A.loff[blk + 1], A.list_cap);   // wave-uniform
        for (uint32_t c0 = s0; c0 < s1; c0 += dev::kWave) {
            const uint32_t e = c0 + (uint32_t)lane;
            const int32_t f = e < s1 ? A.list[e] : -1;
            round(f >= 0 && f < A.faces.F, f, nullptr);
        }
    } else {
        for_candidates(A.bins, bx.ilo, bx.ihi, [&](bool has, int32_t f, const int cur[3]) -> bool {
            round(has, f, cur);
            return true;
        });
    }
    return count;
}

// One wave: finest-level blocks first .. first + 64/4^D - 1 of A; best hit
// per (cell, direction) and the node rows.  out.rows(blk, count) places each
// block's nodes: it returns the first row for them (and records the count),
// or -1 when it has no room; rows are written in cell order.
template <int D, int Q, class Out>
__device__ __forceinline__ void links_wave(const LinkArgs<D, Q> &A, int64_t first, Out &out) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int BPW = 64 / CELLS;
    constexpr int NP = (Q - 1) / 2;            // direction pairs
    __shared__ LinkStaged<D> S;
    __shared__ float s_dir[NP][3];   // D = c * dx of each direction pair's first direction
    const int lane = threadIdx.x;
    if (lane < NP)
        for (int a = 0; a < 3; ++a) s_dir[lane][a] = (float)dir_c<D>(1 + 2 * lane, a) * A.dx[a];
    const int64_t blk = first + lane / CELLS;
    const bool valid = blk < A.n;
    const int cell = lane % CELLS;
    const int sub = lane / CELLS;
    int bc[3] = {0, 0, 0};
    uint32_t key = 0;
    if (valid) {
        key = A.keys[blk];
        dev::decode_key<D>(key, A.level, A.R[0], A.R[1], bc);
    }
    float o[3];
    o[0] = dev::cell_centre(A.lo[0], 4 * bc[0] + (cell & 3), A.dx[0]);
    o[1] = dev::cell_centre(A.lo[1], 4 * bc[1] + ((cell >> 2) & 3), A.dx[1]);
    o[2] = D == 3 ? dev::cell_centre(A.lo[2], 4 * bc[2] + (cell >> 4), A.dx[2]) : 0.0f;
    // Near test of a staged face against the lane's link box (cell +- one cell
    // per axis), separable by axis: a staged face carries one bit per (axis,
    // position) of the block it was staged for, from the same FP32 expressions
    // every lane would use, and a lane tests it with one AND against its own D
    // bits.  (2D: block t of the wave uses bits 8t..8t+7; a face near a cell of
    // block t lies in block t's link box, so it is staged, and coded, for t.)
    const int pos3[3] = {cell & 3, (cell >> 2) & 3, cell >> 4};
    uint32_t lbits = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) lbits |= 1u << (sub * 4 * D + 4 * a + pos3[a]);

    // Best hit per (lane, direction) as one 64-bit key: the FP32 bits of t
    // (t >= 0, so they order like t) above the face id, so the smaller key is
    // the smaller t and, between equal t, the lower face id.
    __shared__ unsigned long long s_best[Q - 1][64];
    __shared__ float s_o[64][3];
    // Work waits in two queues and is taken 64 at a time, one item per lane,
    // whichever lanes queued it: (lane, staged face) pairs for the FP32
    // filter, then (lane, staged face, direction pair) for the FP64 decision.
    constexpr int TCAP = 128;   // below 64 after a take, at most 64 added per step
    __shared__ uint32_t s_qa[TCAP];
    __shared__ uint32_t s_qb[TCAP];
#pragma unroll
    for (int i = 0; i < Q - 1; ++i) s_best[i][lane] = ~0ull;
#pragma unroll
    for (int a = 0; a < 3; ++a) s_o[lane][a] = o[a];
    int na = 0, nb = 0;   // wave-uniform queue lengths

    // A hit at t64 for direction i of lane l.  t is decided in FP64 and kept
    // rounded to FP32 (a negative zero as zero).
    auto consider = [&](int i, int l, double t64, int32_t f) {
        if (!(t64 >= 0.0 && t64 <= 1.0)) return;
        const float t = (float)t64 + 0.0f;
        const unsigned long long k = ((unsigned long long)__float_as_uint(t) << 32) | (uint32_t)f;
        atomicMin(&s_best[i][l], k);
    };
    auto take_b = [&](int take) {   // wave-uniform
        __syncthreads();
        const uint32_t item = lane < take ? s_qb[lane] : 0u;
        __syncthreads();
        if (lane < nb - take) s_qb[lane] = s_qb[take + lane];
        nb -= take;
        if (lane < take) {
            const int l = (int)(item >> 20);
            const int j = (int)((item >> 13) & 127u);
            const int p = (int)(item & 31u);
            const double ol[3] = {s_o[l][0], s_o[l][1], s_o[l][2]};
            const double t = link_decide<D>(S, j, ol, s_dir[p]);
            consider(2 * p, l, t, S.id[j]);        // direction 1 + 2p
            consider(2 * p + 1, l, -t, S.id[j]);   // its opposite
        }
    };
    auto take_a = [&](int take) {   // wave-uniform
        __syncthreads();
        const uint32_t item = lane < take ? s_qa[lane] : 0u;
        __syncthreads();
        if (lane < na - take) s_qa[lane] = s_qa[take + lane];
        na -= take;
        const int l = (int)(item >> 7), j = (int)(item & 127u);
        uint32_t cm = 0;
        if (lane < take) {
            const float ol[3] = {s_o[l][0], s_o[l][1], s_o[l][2]};
            cm = link_filter<D, NP, false, kLinkCap>(S, j, ol, A.dx, nullptr);
        }
        while (__ballot(cm != 0)) {
            const bool has = cm != 0;
            int p = 0;
            if (has) {
                p = __builtin_ctz(cm);
                cm &= cm - 1u;
            }
            const uint64_t m = __ballot(has);
            if (has) s_qb[nb + dev::lanes_below(m)] = ((uint32_t)l << 20) | ((uint32_t)j << 13) | (uint32_t)p;
            nb += __popcll(m);
            if (nb >= 64) take_b(64);
        }
    };

    // Staged faces are visited in batches of 64: each lane marks the faces
    // whose box meets its link box (broadcast LDS reads), then queues its own
    // marked faces that its links can reach.  Both queues are emptied before
    // the staging area is refilled.
    auto test_staged = [&](int n) {
        __syncthreads();
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int jn = min(64, n - j0);
            uint64_t nm = 0;
            if (valid)
            for (int jj = 0; jj < jn; jj += 4) {
                const uint32_t cs[4] = {S.code[j0 + jj], S.code[j0 + jj + 1], S.code[j0 + jj + 2],
                                        S.code[j0 + jj + 3]};
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    nm |= ((cs[u] & lbits) == lbits && jj + u < jn) ? (1ull << (jj + u)) : 0ull;
            }
            while (__ballot(nm != 0)) {
                bool pass = false;
                int j = 0;
                if (nm) {
                    j = j0 + __builtin_ctzll(nm);
                    nm &= nm - 1ull;
                    pass = link_reach<D>(S, j, o, A.dx);
                }
                const uint64_t m = __ballot(pass);
                if (pass) s_qa[na + dev::lanes_below(m)] = ((uint32_t)lane << 7) | (uint32_t)j;
                na += __popcll(m);
                if (na >= 64) take_a(64);
            }
        }
        if (na > 0) take_a(na);
        if (nb > 0) take_b(nb);
        __syncthreads();
    };

    int count = 0;
    for (int sb = 0; sb < BPW; ++sb) {
        if (first + sb >= A.n) break;
        int sc[3];
        sc[0] = __shfl(bc[0], sb * CELLS, 64);
        sc[1] = __shfl(bc[1], sb * CELLS, 64);
        sc[2] = __shfl(bc[2], sb * CELLS, 64);
        LinkBox<D> bx;
        link_box<D, Q>(A, sc, bx);
        count = link_gather<D, Q>(A, first + sb, sb, bx, S, count, test_staged);
    }
    if (count > 0) test_staged(count);

    uint64_t best[Q - 1];
    bool has = false;
#pragma unroll
    for (int i = 0; i < Q - 1; ++i) {
        best[i] = s_best[i][lane];
        has = has || best[i] != ~0ull;
    }
    // ordered compaction of the cells that have a link
    has = has && valid;
    const uint64_t hm = __ballot(has);
    // rank inside the block: lanes of this block below this lane that have a link
    uint64_t bm = hm;
    if constexpr (CELLS < 64) bm = (hm >> (sub * CELLS)) & ((1ull << CELLS) - 1);
    int64_t row0 = 0;
    if (valid && cell == 0) row0 = out.rows(blk, (uint32_t)__popcll(bm));
    row0 = __shfl(row0, sub * CELLS, 64);
    // a negative first row: the output policy ran out of capacity
    const int64_t node = has && row0 >= 0 ? row0 + __popcll(bm & ((1ull << cell) - 1)) : -1;
    if (node >= 0) {
        A.node_key[node] = (uint64_t)key * CELLS + (uint64_t)cell;
        float *qr = A.q + node * Q;
        int32_t *fr = A.face + node * Q;
        qr[0] = -1.0f;
        fr[0] = -1;
#pragma unroll
        for (int i = 0; i < Q - 1; ++i) {
            const bool hit = best[i] != ~0ull;
            qr[i + 1] = hit ? __uint_as_float((uint32_t)(best[i] >> 32)) : -1.0f;
            fr[i + 1] = hit ? (int32_t)(uint32_t)best[i] : -1;
        }
    }
}

// Near code of a face box bb (min[D], max[D]) for the block at block
// coordinates bc: bit 4a + i is set when the link box of cell position i along
// axis a (centre +- one cell, widened by eps) meets the box along a -- the
// same FP32 expressions as link_box.  Per lane (the block need not be
// wave-uniform).
template <int D, int Q>
__device__ __forceinline__ uint32_t link_code_at(const LinkArgs<D, Q> &A, const int bc[3], const float *bb) {
    uint32_t c = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float m = dev::cell_centre(A.lo[a], 4 * bc[a] + i, A.dx[a]);
            const float lo_ = (m - A.dx[a]) - A.eps[a], hi_ = (m + A.dx[a]) + A.eps[a];
            c |= (bb[a] <= hi_ && bb[D + a] >= lo_) ? (1u << (4 * a + i)) : 0u;
        }
    return c;
}

// The set bits of a 4-bit mask in ascending order, two bits each (entry k
// of the list is (list >> 2k) & 3).
__device__ __forceinline__ uint32_t bit_list4(uint32_t m) {
    uint32_t list = 0, n = 0;
#pragma unroll
    for (uint32_t b = 0; b < 4; ++b)
        if ((m >> b) & 1u) {
            list |= b << (2 * n);
            ++n;
        }
    return list;
}

// u / n for n in 1 .. 4 and u < 4096 as (u * 2^16 / n) >> 16 (exact there:
// the multiplier for 3 is 2^16 / 3 rounded up, off by less than 2^-16 of u).
__device__ __forceinline__ uint32_t div_1to4(uint32_t u, uint32_t n) {
    return (u * (n == 3u ? 21846u : 65536u >> (n >> 1))) >> 16;
}

// Node pass of list mode: which finest-level cells have at least one link.
// Work is taken from the candidate lists 64 (face, block) entries at a time
// (persistent loop over the entries): every (entry, cell) pair whose cell
// link box meets the face box -- exactly the pairs the row pass tests -- is
// one lane's work.  A pair is dropped when its cell is known to have a link
// already or when no direction can reach the face's plane; the others go
// through a queue, 64 at a time, to the FP32 filter narrowed and widened by
// its margins: a certain hit sets the cell's bit in its block's mask, a
// possible one is decided in FP64 exactly as the row pass decides it.  So a
// block's mask is the set of its cells for which the row pass finds a hit.
// The 64 entries of a window belong to a few blocks (the lists are in block
// order): each block's mask is read once into LDS, hits are ORed there, and
// the new bits go out with one device atomic per block at the window's end
// (device-scope atomics are performed past the per-XCD L2, so one per hit
// costs memory-side traffic).
// mask: one 64-bit word per block, zeroed; lblk: the block of each entry.
template <int D, int Q>
__device__ __forceinline__ void links_nodes_entries(const LinkArgs<D, Q> &A, const uint32_t *lblk,
                                                    unsigned long long *mask, int64_t wg, int64_t nwg) {
    constexpr int NP = (Q - 1) / 2;
    constexpr int RF = dev::kRecFloats<D>;
    __shared__ LinkStaged<D, 64> S;
    __shared__ float s_dir[NP][3];
    __shared__ uint32_t s_pre[64];     // exclusive prefix of the entries' pair counts
    __shared__ uint32_t s_enum[64];    // each entry's cells per axis: bit lists x, y, z and counts
    __shared__ int s_bc[64][3];        // its block coordinates
    __shared__ uint32_t s_head[64];    // first entry of the window with the same block
    __shared__ unsigned long long s_m[64];   // at a block's first entry: its mask as known to the wave
    constexpr int QCAP = 128;
    __shared__ uint32_t s_q[QCAP];     // queued pairs: entry << 8 | cell
    const int lane = dev::lane_id();
    if (lane < NP)
        for (int a = 0; a < 3; ++a) s_dir[lane][a] = (float)dir_c<D>(1 + 2 * lane, a) * A.dx[a];
    const uint32_t total = min(A.loff[A.n], A.list_cap);
    int nq = 0;   // wave-uniform queue length

    for (int64_t w = wg; w * 64 < (int64_t)total; w += nwg) {
        const uint32_t e = (uint32_t)(w * 64) + (uint32_t)lane;
        uint32_t bits = 0, cnt = 0, b = 0;
        int bc[3] = {0, 0, 0};
        if (e < total) {
            const int32_t f = A.list[e];
            b = lblk[e];
            if (f >= 0 && f < A.faces.F && (int64_t)b < A.n) {
                float r[RF];
                dev::load_rec<D>(A.faces.rec, f, r);
                dev::decode_key<D>(A.keys[b], A.level, A.R[0], A.R[1], bc);
                bits = link_code_at<D, Q>(A, bc, r + D * D);
                cnt = 1;
#pragma unroll
                for (int a = 0; a < D; ++a) cnt *= (uint32_t)__popc((bits >> (4 * a)) & 15u);
                link_stage<D>(S, lane, f, r, A.dx, bits);
            }
        }
        const uint32_t incl = dev::wave_inclusive_sum(cnt);
        const uint32_t npairs = (uint32_t)__builtin_amdgcn_readlane((int)incl, dev::kWave - 1);
        s_pre[lane] = incl - cnt;
        {
            const uint32_t mx = bits & 15u, my = (bits >> 4) & 15u, mz = (bits >> 8) & 15u;
            const uint32_t nx = (uint32_t)__popc(mx), ny = (uint32_t)__popc(my);
            // bit lists (8 bits each) and the x and y counts less one (2 bits each)
            s_enum[lane] = cnt ? (bit_list4(mx) | (bit_list4(my) << 8) | (bit_list4(mz) << 16) | ((nx - 1u) << 24) |
                                  ((D == 3 ? ny - 1u : 0u) << 26))
                               : 0u;
        }
        s_bc[lane][0] = bc[0];
        s_bc[lane][1] = bc[1];
        s_bc[lane][2] = bc[2];
        const bool live = e < total && (int64_t)b < A.n;
        const uint32_t prev_b = (uint32_t)__shfl_up((int)b, 1, dev::kWave);
        const bool head = live && (lane == 0 || prev_b != b);
        const uint64_t heads = __ballot(head);
        const uint64_t upto = lane == dev::kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
        const uint64_t hb = heads & upto;
        s_head[lane] = hb ? (uint32_t)(63 - __clzll((long long)hb)) : (uint32_t)lane;
        const unsigned long long m0 = head ? mask[b] : 0ull;
        s_m[lane] = m0;
        dev::wave_sync();
        // one work loop: enumerate 64 pairs, queueing those still open, and
        // decide 64 queued pairs whenever the queue holds that many (or the
        // pairs are exhausted); each step has one place in the code
        uint32_t c0 = 0;
        while (true) {
            if (nq >= 64 || (nq > 0 && c0 >= npairs)) {
                const int ntake = min(nq, 64);
                dev::wave_sync();
                const uint32_t item = lane < ntake ? s_q[lane] : 0u;
                dev::wave_sync();
                if (lane < nq - ntake) s_q[lane] = s_q[ntake + lane];
                nq -= ntake;
                if (lane < ntake) {
                    const int j = (int)(item >> 8), cell = (int)(item & 255u);
                    float o[3] = {0.0f, 0.0f, 0.0f};
                    o[0] = dev::cell_centre(A.lo[0], 4 * s_bc[j][0] + (cell & 3), A.dx[0]);
                    o[1] = dev::cell_centre(A.lo[1], 4 * s_bc[j][1] + ((cell >> 2) & 3), A.dx[1]);
                    if constexpr (D == 3) o[2] = dev::cell_centre(A.lo[2], 4 * s_bc[j][2] + (cell >> 4), A.dx[2]);
                    bool hit = false;
                    uint32_t maybe = link_filter<D, NP, true, 64>(S, j, o, A.dx, &hit);
                    if (!hit && maybe) {
                        const double o64[3] = {o[0], o[1], o[2]};
                        while (maybe) {
                            const int p = __builtin_ctz(maybe);
                            maybe &= maybe - 1u;
                            const double t = link_decide<D>(S, j, o64, s_dir[p]);
                            if (t >= -1.0 && t <= 1.0) {
                                hit = true;
                                break;
                            }
                        }
                    }
                    if (hit) atomicOr(&s_m[s_head[j]], 1ull << cell);
                }
            } else if (c0 < npairs) {
                const uint32_t v = c0 + (uint32_t)lane;
                c0 += dev::kWave;
                bool want = false;
                uint32_t item = 0;
                if (v < npairs) {
                    int k = 0;   // the last entry whose pairs start at or before v
#pragma unroll
                    for (int step = 32; step >= 1; step >>= 1)
                        if (s_pre[k + step] <= v) k += step;
                    // pair u of entry k: x fastest, then y, then z over the entry's cells
                    const uint32_t u = v - s_pre[k];
                    const uint32_t en = s_enum[k];
                    const uint32_t nx = ((en >> 24) & 3u) + 1u, ny = ((en >> 26) & 3u) + 1u;
                    const uint32_t q1 = div_1to4(u, nx);
                    const uint32_t ux = u - q1 * nx;
                    uint32_t uy = q1, uz = 0;
                    if constexpr (D == 3) {
                        uz = div_1to4(q1, ny);
                        uy = q1 - uz * ny;
                    }
                    const int ix = (int)((en >> (2 * ux)) & 3u);
                    const int iy = (int)((en >> (8 + 2 * uy)) & 3u);
                    const int iz = D == 3 ? (int)((en >> (16 + 2 * uz)) & 3u) : 0;
                    const int cell = ix | (iy << 2) | (iz << 4);
                    if (!((s_m[s_head[k]] >> cell) & 1ull)) {
                        float o[3] = {0.0f, 0.0f, 0.0f};
                        o[0] = dev::cell_centre(A.lo[0], 4 * s_bc[k][0] + ix, A.dx[0]);
                        o[1] = dev::cell_centre(A.lo[1], 4 * s_bc[k][1] + iy, A.dx[1]);
                        if constexpr (D == 3) o[2] = dev::cell_centre(A.lo[2], 4 * s_bc[k][2] + iz, A.dx[2]);
                        want = link_reach<D>(S, k, o, A.dx);
                        item = ((uint32_t)k << 8) | (uint32_t)cell;
                    }
                }
                const uint64_t m = __ballot(want);
                if (want) s_q[nq + dev::lanes_below(m)] = item;
                nq += __popcll(m);
            } else {
                break;
            }
        }
        dev::wave_sync();
        if (head) {
            const unsigned long long m1 = s_m[lane];
            if (m1 != m0) atomicOr(&mask[b], m1 & ~m0);
        }
        dev::wave_sync();
    }
}

// Row pass of list mode: one wave per kRowNodes consecutive nodes (node k:
// block nblk[k], node key written beforehand), one lane per node.  28 nodes
// per wave keep the best-key table at 5.8 KB and the wave's LDS at 8.75 KB, so
// that 18 waves fit a CU (64 nodes: 9 waves and 14 % slower; 16, 20, 24, 32
// and 48 measured too: fewer nodes per wave stage the same entries more often,
// which costs more than the extra waves gain).
// kRowNodes * Q words stay a multiple of four for the 16-byte row stores.  The wave stages
// the candidate entries of its blocks -- one contiguous range of the lists,
// blocks being in node order -- and every lane tests the staged faces of its
// own block near its cell; the best hit per direction is kept as in
// links_wave, in a node-major table from which the wave writes its rows of q
// and face ids as flat coalesced runs.
constexpr int kRowNodes = 28;   // nodes per wave of the row pass
static_assert(kRowNodes % 4 == 0 && kRowNodes <= 64, "16-byte row stores, one lane per node");

template <int D, int Q>
__device__ __forceinline__ void links_rows_nodes(const LinkArgs<D, Q> &A, const uint32_t *lblk, const uint32_t *nblk,
                                                 const uint64_t *node_key, uint32_t nn, int64_t chunk) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int NP = (Q - 1) / 2;
    constexpr int RF = dev::kRecFloats<D>;
    __shared__ LinkStaged<D, kLinkCap, false> S;
    __shared__ uint32_t s_sblk[kLinkCap];   // block of each staged entry
    __shared__ float s_dir[NP][3];
    static_assert(kLinkCap <= 32 && kRowNodes <= 32 && NP <= 32, "near masks are 32-bit; queue items 16-bit");
    const int lane = dev::lane_id();
    if (lane < NP)
        for (int a = 0; a < 3; ++a) s_dir[lane][a] = (float)dir_c<D>(1 + 2 * lane, a) * A.dx[a];
    const int64_t k0 = chunk * kRowNodes;
    const int nnodes = (int)min<int64_t>(kRowNodes, (int64_t)nn - k0);
    const bool valid = lane < nnodes;
    const uint32_t myb = valid ? nblk[k0 + lane] : 0xFFFFFFFFu;
    const uint64_t nkey = valid ? node_key[k0 + lane] : 0ull;
    const int cell = (int)(nkey % CELLS);
    int bc[3] = {0, 0, 0};
    if (valid) dev::decode_key<D>((uint32_t)(nkey / CELLS), A.level, A.R[0], A.R[1], bc);
    float o[3];
    o[0] = dev::cell_centre(A.lo[0], 4 * bc[0] + (cell & 3), A.dx[0]);
    o[1] = dev::cell_centre(A.lo[1], 4 * bc[1] + ((cell >> 2) & 3), A.dx[1]);
    o[2] = D == 3 ? dev::cell_centre(A.lo[2], 4 * bc[2] + (cell >> 4), A.dx[2]) : 0.0f;
    uint32_t lbits = 0;
    {
        const int pos3[3] = {cell & 3, (cell >> 2) & 3, cell >> 4};
#pragma unroll
        for (int a = 0; a < D; ++a) lbits |= 1u << (4 * a + pos3[a]);
    }
    // node-major best keys: a row of Q - 1 keys per node, read back in row order
    __shared__ unsigned long long s_best[kRowNodes][Q - 1];
    __shared__ float s_o[kRowNodes][3];
    constexpr int TCAP = 128;
    __shared__ uint16_t s_qa[TCAP];   // (node, staged entry) pairs to filter: l << 5 | j
    __shared__ uint16_t s_qb[TCAP];   // direction pairs to decide: l << 10 | j << 5 | p
    if (lane < kRowNodes) {
#pragma unroll
        for (int i = 0; i < Q - 1; ++i) s_best[lane][i] = ~0ull;
#pragma unroll
        for (int a = 0; a < 3; ++a) s_o[lane][a] = o[a];
    }
    int na = 0, nb = 0;

    auto consider = [&](int i, int l, double t64, int32_t f) {
        if (!(t64 >= 0.0 && t64 <= 1.0)) return;
        const float t = (float)t64 + 0.0f;
        const unsigned long long key = ((unsigned long long)__float_as_uint(t) << 32) | (uint32_t)f;
        atomicMin(&s_best[l][i], key);
    };
    auto take_b = [&](int take) {
        dev::wave_sync();
        const uint32_t item = lane < take ? (uint32_t)s_qb[lane] : 0u;
        dev::wave_sync();
        if (lane < nb - take) s_qb[lane] = s_qb[take + lane];
        nb -= take;
        if (lane < take) {
            const int l = (int)(item >> 10);
            const int j = (int)((item >> 5) & 31u);
            const int p = (int)(item & 31u);
            const double ol[3] = {s_o[l][0], s_o[l][1], s_o[l][2]};
            const double t = link_decide<D>(S, j, ol, s_dir[p]);
            consider(2 * p, l, t, S.id[j]);
            consider(2 * p + 1, l, -t, S.id[j]);
        }
    };
    auto take_a = [&](int take) {
        dev::wave_sync();
        const uint32_t item = lane < take ? (uint32_t)s_qa[lane] : 0u;
        dev::wave_sync();
        if (lane < na - take) s_qa[lane] = s_qa[take + lane];
        na -= take;
        const int l = (int)(item >> 5), j = (int)(item & 31u);
        uint32_t cm = 0;
        if (lane < take) {
            const float ol[3] = {s_o[l][0], s_o[l][1], s_o[l][2]};
            cm = link_filter<D, NP, false, kLinkCap>(S, j, ol, A.dx, nullptr);
        }
        while (__ballot(cm != 0)) {
            const bool has = cm != 0;
            int p = 0;
            if (has) {
                p = __builtin_ctz(cm);
                cm &= cm - 1u;
            }
            const uint64_t m = __ballot(has);
            if (has) s_qb[nb + dev::lanes_below(m)] = (uint16_t)((l << 10) | (j << 5) | p);
            nb += __popcll(m);
            if (nb >= 64) take_b(64);
        }
    };
    // staged entries near the lane's cell (same block, all its code bits),
    // queued while its links can reach them; both queues emptied before the
    // staging area is refilled
    auto test_staged = [&](int n) {
        dev::wave_sync();
        uint32_t nm = 0;
        if (valid) {
            // staged entries keep the lists' block order: the lane's own block is one range, found by two
            // binary searches, and only that range is tested
            int lo = 0, hi = n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_sblk[mid] < myb) lo = mid + 1;
                else hi = mid;
            }
            const int jlo = lo;
            hi = n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_sblk[mid] <= myb) lo = mid + 1;
                else hi = mid;
            }
            for (int j = jlo; j < lo; ++j) nm |= ((S.code[j] & lbits) == lbits) ? (1u << j) : 0u;
        }
        while (__ballot(nm != 0)) {
            bool pass = false;
            int j = 0;
            if (nm) {
                j = __builtin_ctz(nm);
                nm &= nm - 1u;
                pass = link_reach<D>(S, j, o, A.dx);
            }
            const uint64_t m = __ballot(pass);
            if (pass) s_qa[na + dev::lanes_below(m)] = (uint16_t)((lane << 5) | j);
            na += __popcll(m);
            if (na >= 64) take_a(64);
        }
        if (na > 0) take_a(na);
        if (nb > 0) take_b(nb);
        dev::wave_sync();
    };

    // the wave's entries: lists of blocks nblk[k0] .. nblk[k0 + nnodes - 1]
    const uint32_t b_first = (uint32_t)__builtin_amdgcn_readfirstlane((int)nblk[k0]);
    const uint32_t b_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)nblk[k0 + nnodes - 1]);
    const uint32_t e0 = A.loff[b_first], e1 = min(A.loff[b_last + 1], A.list_cap);
    int count = 0;
    for (uint32_t c0 = e0; c0 < e1; c0 += dev::kWave) {
        const uint32_t e = c0 + (uint32_t)lane;
        bool keep = false;
        int32_t f = -1;
        uint32_t b = 0, code = 0;
        float r[RF];
        if (e < e1) {
            f = A.list[e];
            b = lblk[e];
            if (f >= 0 && f < A.faces.F && (int64_t)b < A.n) {
                dev::load_rec<D>(A.faces.rec, f, r);
                int ebc[3] = {0, 0, 0};
                dev::decode_key<D>(A.keys[b], A.level, A.R[0], A.R[1], ebc);
                code = link_code_at<D, Q>(A, ebc, r + D * D);
                keep = true;
#pragma unroll
                for (int a = 0; a < D; ++a) keep = keep && ((code >> (4 * a)) & 15u) != 0u;
            }
        }
        uint64_t rest = __ballot(keep);
        while (rest) {
            if (count > 0 && count + __popcll(rest) > kLinkCap) {
                test_staged(count);
                count = 0;
            }
            const bool now = ((rest >> lane) & 1ull) && dev::lanes_below(rest) < kLinkCap - count;
            const uint64_t part = __ballot(now);
            rest &= ~part;
            const int pos = count + dev::lanes_below(part);
            count += __popcll(part);
            if (now) {
                link_stage<D>(S, pos, f, r, A.dx, code);
                s_sblk[pos] = b;
            }
        }
    }
    if (count > 0) test_staged(count);
    dev::wave_sync();

    // rows k0 .. k0 + nnodes - 1 of q and face ids: element e of the span is
    // node e / Q, direction e % Q.  Each lane writes four consecutive elements
    // with 16-byte stores (the span starts on a 16-byte boundary: kRowNodes Q
    // words per wave), the last few elements one at a time.
    float *qd = A.q + k0 * Q;
    int32_t *fd = A.face + k0 * Q;
    const int total = nnodes * Q, total4 = total & ~3;
    int l = (4 * lane) / Q, i = (4 * lane) % Q;   // node and direction of element 4 lane, advanced 256 a step
    for (int e = 4 * lane; e < total4; e += 256) {
        float qv[4];
        int32_t fv[4];
        int ll = l, ii = i;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned long long key = ii == 0 ? ~0ull : s_best[ll][ii - 1];
            const bool hit = key != ~0ull;
            qv[k] = hit ? __uint_as_float((uint32_t)(key >> 32)) : -1.0f;
            fv[k] = hit ? (int32_t)(uint32_t)key : -1;
            if (++ii == Q) {
                ii = 0;
                ++ll;
            }
        }
        // rows are not read again by this pass: stored past the caches' keep policy
        typedef float f4 __attribute__((ext_vector_type(4)));
        typedef int i4 __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(f4{qv[0], qv[1], qv[2], qv[3]}, reinterpret_cast<f4 *>(qd + e));
        __builtin_nontemporal_store(i4{fv[0], fv[1], fv[2], fv[3]}, reinterpret_cast<i4 *>(fd + e));
        i += 256 % Q;
        l += 256 / Q;
        if (i >= Q) {
            i -= Q;
            ++l;
        }
    }
    if (lane < total - total4) {
        const int e = total4 + lane;
        const int le = e / Q, ie = e % Q;
        const unsigned long long key = ie == 0 ? ~0ull : s_best[le][ie - 1];
        const bool hit = key != ~0ull;
        qd[e] = hit ? __uint_as_float((uint32_t)(key >> 32)) : -1.0f;
        fd[e] = hit ? (int32_t)(uint32_t)key : -1;
    }
}

// ---------------------------------------------------------------------------
// Adjoint: a queue of live links per tile of nodes, one link per thread.
// ---------------------------------------------------------------------------
template <int D, int Q>
struct AdjArgs {
    const float *rec;      // face records (F x kRecFloats<D>)
    int64_t F;
    const int32_t *fidx;
    const uint64_t *node_key;
    const int32_t *face;
    const float *gq;
    int64_t n;
    int level;
    int R[3];
    float lo[3];
    float dx[3];
    float *grad;
};

constexpr int kAdjThreads = 256;   // nodes per tile = threads per workgroup
constexpr int kAdjWaves = kAdjThreads / 64;
constexpr int kAdjGroup = 4;      // slots per lane per wave step (queued between takes: up to 64 x this)
constexpr int kAdjHashBits = 9;
constexpr int kAdjHash = 1 << kAdjHashBits;   // per-workgroup face accumulators

// Gradient of one link's t with respect to the D vertices of its face, scaled
// by the link's weight w: out[k][a] = s_k n_a with s_k = w lambda_k / (D . n),
// lambda the barycentric coordinates of the hit and n = E1 x E2 (2D: the edge
// normal).  n belongs to the face, so the links of one face are summed as the
// D scalars s_k and multiplied by n once.
//
// face_normal is the one expression of n (per link and at the final scatter).
// link_setup sets up what depends on the face and the node only (edges,
// normal, cross products with T = o - v0); link_scalars adds the direction.
// A grazing link (|D . n| below 2^-10 of |D| |E1| |E2|) takes its barycentrics
// and denominator in FP64 from the FP32 data.
template <int D>
__device__ __forceinline__ void face_normal(const float *v, float n[3]) {
    if constexpr (D == 3) {
        const float e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
        const float e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    } else {
        n[0] = -(v[3] - v[1]);
        n[1] = v[2] - v[0];
        n[2] = 0.0f;
    }
}

template <int D>
struct LinkFace {
    float v[dev::kRecFloats<D>];               // the face record
    float e1[3], e2[3], n[3], p1[3], p2[3];   // 3D: edges, normal, T x E2, E1 x T   (T = o - v0)
    float ee;                                  // |E1| |E2| (2D: |E|)
};

template <int D>
__device__ __forceinline__ void link_setup(const float *rec, int32_t f, const float o[3], LinkFace<D> &R) {
    dev::load_rec<D>(rec, f, R.v);
    const float *v = R.v;
    face_normal<D>(v, R.n);
    if constexpr (D == 3) {
        const float e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
        const float e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
        const float T[3] = {o[0] - v[0], o[1] - v[1], o[2] - v[2]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R.e1[a] = e1[a];
            R.e2[a] = e2[a];
        }
        R.p1[0] = T[1] * e2[2] - T[2] * e2[1];
        R.p1[1] = T[2] * e2[0] - T[0] * e2[2];
        R.p1[2] = T[0] * e2[1] - T[1] * e2[0];
        R.p2[0] = e1[1] * T[2] - e1[2] * T[1];
        R.p2[1] = e1[2] * T[0] - e1[0] * T[2];
        R.p2[2] = e1[0] * T[1] - e1[1] * T[0];
        R.ee = sqrtf((e1[0] * e1[0] + e1[1] * e1[1]) + e1[2] * e1[2]) *
               sqrtf((e2[0] * e2[0] + e2[1] * e2[1]) + e2[2] * e2[2]);
    } else {
        const float e0 = v[2] - v[0], e1 = v[3] - v[1];
        R.e1[0] = e0;
        R.e1[1] = e1;
        R.p1[0] = v[0] - o[0];   // w = a - o
        R.p1[1] = v[1] - o[1];
        R.ee = sqrtf(e0 * e0 + e1 * e1);
    }
}

// Link of direction Dv (length dd) with weight w: s[k] = w * lambda_k / (D . n).
template <int D>
__device__ __forceinline__ void link_scalars(const float o[3], const LinkFace<D> &R, const float Dv[3], float dd,
                                             float w, float s[D]) {
    float lam[D], inv;
    const float *v = R.v;
    if constexpr (D == 3) {
        const float den = (Dv[0] * R.n[0] + Dv[1] * R.n[1]) + Dv[2] * R.n[2];
        float u, vv;
        if (fabsf(den) < 0.0009765625f * dd * R.ee) {
            double E1[3], E2[3], N[3], TT[3];
            for (int a = 0; a < 3; ++a) {
                E1[a] = (double)v[3 + a] - (double)v[a];
                E2[a] = (double)v[6 + a] - (double)v[a];
                TT[a] = (double)o[a] - (double)v[a];
            }
            N[0] = E1[1] * E2[2] - E1[2] * E2[1];
            N[1] = E1[2] * E2[0] - E1[0] * E2[2];
            N[2] = E1[0] * E2[1] - E1[1] * E2[0];
            const double den64 = (double)Dv[0] * N[0] + (double)Dv[1] * N[1] + (double)Dv[2] * N[2];
            const double P1[3] = {TT[1] * E2[2] - TT[2] * E2[1], TT[2] * E2[0] - TT[0] * E2[2],
                                  TT[0] * E2[1] - TT[1] * E2[0]};
            const double P2[3] = {E1[1] * TT[2] - E1[2] * TT[1], E1[2] * TT[0] - E1[0] * TT[2],
                                  E1[0] * TT[1] - E1[1] * TT[0]};
            u = (float)(((double)Dv[0] * P1[0] + (double)Dv[1] * P1[1] + (double)Dv[2] * P1[2]) / den64);
            vv = (float)(((double)Dv[0] * P2[0] + (double)Dv[1] * P2[1] + (double)Dv[2] * P2[2]) / den64);
            inv = (float)(1.0 / den64);
        } else {
            inv = 1.0f / den;
            u = ((Dv[0] * R.p1[0] + Dv[1] * R.p1[1]) + Dv[2] * R.p1[2]) * inv;
            vv = ((Dv[0] * R.p2[0] + Dv[1] * R.p2[1]) + Dv[2] * R.p2[2]) * inv;
        }
        lam[0] = 1.0f - u - vv;
        lam[1] = u;
        lam[2] = vv;
    } else {
        const float e0 = R.e1[0], e1 = R.e1[1];
        const float w0 = R.p1[0], w1 = R.p1[1];
        const float den = Dv[0] * R.n[0] + Dv[1] * R.n[1];
        float sp;
        if (fabsf(den) < 0.0009765625f * dd * R.ee) {
            const double E0 = (double)v[2] - (double)v[0], E1 = (double)v[3] - (double)v[1];
            const double W0 = (double)v[0] - (double)o[0], W1 = (double)v[1] - (double)o[1];
            const double dxe = (double)Dv[0] * E1 - (double)Dv[1] * E0;   // D x e
            sp = (float)((W0 * (double)Dv[1] - W1 * (double)Dv[0]) / dxe);
            inv = (float)(1.0 / ((double)Dv[0] * -E1 + (double)Dv[1] * E0));
        } else {
            const float dxe = Dv[0] * e1 - Dv[1] * e0;
            sp = (w0 * Dv[1] - w1 * Dv[0]) / dxe;
            inv = 1.0f / den;
        }
        lam[0] = 1.0f - sp;
        lam[1] = sp;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) s[k] = w * lam[k] * inv;
}

// s += the DPP-moved s (control CTRL: row_shr:n = 0x110 + n, row_bcast:15 =
// 0x142, row_bcast:31 = 0x143; ROWS: the rows written) on the lanes with use;
// lanes without a source, or in rows not written, move 0.  Every lane active.
template <int CTRL, int ROWS, int N>
__device__ __forceinline__ void dpp_add(float (&s)[N], bool use) {
    float up[N];
#pragma unroll
    for (int k = 0; k < N; ++k)
        up[k] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s[k]), CTRL, ROWS, 0xF, false));
    if (use)
#pragma unroll
        for (int k = 0; k < N; ++k) s[k] += up[k];
}

// Inclusive sum over the wave on DPP (every lane active): row shifts by 1, 2,
// 4 and 8, then lane 15 of the previous row into rows 1 and 3 and lane 31
// into rows 2 and 3; lanes without a source add 0.
__device__ __forceinline__ uint32_t dpp_inclusive_sum(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return v;
}

// The links of a tile of kAdjThreads nodes: the tile's face and weight rows
// are one contiguous span, read kAdjGroup slots per lane with 16-byte loads,
// the waves taking every kAdjWaves-th step of 64 kAdjGroup slots with the
// next step's loads in flight.  Each wave appends the live slots it reads (a
// face and a non-zero weight) to a queue of its own and takes 64 at a time,
// one link per lane, whatever the per-node link counts.  Queue order is slot
// order, so the links of one face tend to sit in neighbouring lanes: a
// segmented sum over runs of equal face ids leaves one lane per run, which
// adds the run's D scalars to the face's entry of the workgroup's LDS hash
// table (neighbouring nodes in key order hit few distinct faces).  At the end
// each face's sums, times its normal, are added per vertex in a second LDS hash
// table (a tile's faces share most of their vertices), and each vertex's sum
// goes out with one float atomic per coordinate: about a sixth of the global
// atomics of sending every face's share straight to its vertices.  One
// workgroup of kAdjThreads threads: nodes node0 .. node0 + kAdjThreads - 1 of A.
template <int D, int Q>
__device__ __forceinline__ void adjoint_tile(const AdjArgs<D, Q> &A, int64_t node0) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int QCAP = (kAdjGroup + 1) * dev::kWave;   // below 64 after the takes, 64 kAdjGroup per step added
    static_assert(Q <= 32, "direction index packed in 5 bits");
    __shared__ int32_t s_key[kAdjHash];
    __shared__ float s_acc[kAdjHash][D];
    __shared__ float s_D[Q][4];   // c_i * dx per axis, then its length
    __shared__ float s_o[kAdjThreads][3];
    // the link queues (tile-local node * 32 + direction, face), reused at the
    // end for the vertex table
    __shared__ uint32_t s_qraw[2 * kAdjWaves * QCAP];
    uint32_t(*s_meta)[QCAP] = reinterpret_cast<uint32_t(*)[QCAP]>(s_qraw);
    int32_t(*s_qf)[QCAP] = reinterpret_cast<int32_t(*)[QCAP]>(s_qraw + kAdjWaves * QCAP);
    constexpr int kVHash = 512;   // vertex accumulators (power of two)
    static_assert(kVHash * (1 + D) <= 2 * kAdjWaves * QCAP, "vertex table fits in the queues");
    int32_t *v_key = reinterpret_cast<int32_t *>(s_qraw);
    float(*v_acc)[D] = reinterpret_cast<float(*)[D]>(s_qraw + kVHash);
    const int tid = threadIdx.x;
    const int lane = dev::lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(tid / dev::kWave);
    for (int i = tid; i < kAdjHash; i += kAdjThreads) {
        s_key[i] = -1;
#pragma unroll
        for (int k = 0; k < D; ++k) s_acc[i][k] = 0.0f;
    }
    if (tid < Q) {
        float d[3];
        for (int a = 0; a < 3; ++a) d[a] = (float)dir_c<D>(tid, a) * A.dx[a];
        for (int a = 0; a < 3; ++a) s_D[tid][a] = d[a];
        s_D[tid][3] = D == 3 ? sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) : sqrtf(d[0] * d[0] + d[1] * d[1]);
    }
    const int nn = (int)min((int64_t)kAdjThreads, A.n - node0);
    if (tid < nn) {
        const uint64_t nk = A.node_key[node0 + tid];
        const uint32_t key = (uint32_t)(nk / CELLS);
        const int cell = (int)(nk % CELLS);
        int bc[3];
        dev::decode_key<D>(key, A.level, A.R[0], A.R[1], bc);
        s_o[tid][0] = dev::cell_centre(A.lo[0], 4 * bc[0] + (cell & 3), A.dx[0]);
        s_o[tid][1] = dev::cell_centre(A.lo[1], 4 * bc[1] + ((cell >> 2) & 3), A.dx[1]);
        s_o[tid][2] = D == 3 ? dev::cell_centre(A.lo[2], 4 * bc[2] + (cell >> 4), A.dx[2]) : 0.0f;
    }
    __syncthreads();

    // Scalars s of face f (normal n) into the hash table; a full table sends
    // s_k n straight to the vertices.
    auto to_lds = [&](int32_t f, const float (&s)[D], const float (&n)[3]) {
        uint32_t h = ((uint32_t)f * 2654435761u) >> (32 - kAdjHashBits);
        for (int probe = 0; probe < kAdjHash; ++probe) {
            const int32_t prev = atomicCAS(&s_key[h], -1, f);
            if (prev == -1 || prev == f) {
#pragma unroll
                for (int k = 0; k < D; ++k) atomicAdd(&s_acc[h][k], s[k]);
                return;
            }
            h = (h + 1) & (kAdjHash - 1);
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int64_t vk = A.fidx[(int64_t)f * D + k];
#pragma unroll
            for (int a = 0; a < D; ++a) unsafeAtomicAdd(&A.grad[vk * D + a], s[k] * n[a]);
        }
    };
    uint32_t *qm = s_meta[wv];
    int32_t *qf = s_qf[wv];
    const int64_t base = node0 * Q;
    int qn = 0;   // wave-uniform queue length
    // Takes queue entries 0 .. take-1 (one per lane), moves the rest to the
    // front, computes the taken links and sums them per run of equal faces.
    auto take = [&](int cnt) {
        dev::wave_sync();
        const int t = min(cnt, dev::kWave);
        uint32_t meta = 0;
        int32_t f = -1;
        if (lane < t) {
            meta = qm[lane];
            f = qf[lane];
        }
        dev::wave_sync();
        // up to 4 x 64 entries remain: every lane moves several, in order (a
        // read of entry t + i precedes the write of entry i + 64 over it)
        for (int i = lane; i < cnt - t; i += dev::kWave) {
            qm[i] = qm[t + i];
            qf[i] = qf[t + i];
        }
        qn = cnt - t;
        float s[D], n[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < D; ++k) s[k] = 0.0f;
        if (lane < t) {
            const int nl = (int)(meta >> 5), i = (int)(meta & 31u);
            const float w = A.gq[base + nl * Q + i];   // read again (just fetched): keeps queue entries at 8 B
            const float o[3] = {s_o[nl][0], s_o[nl][1], s_o[nl][2]};
            const float Dv[3] = {s_D[i][0], s_D[i][1], s_D[i][2]};
            LinkFace<D> R;
            link_setup<D>(A.rec, f, o, R);
            link_scalars<D>(o, R, Dv, s_D[i][3], w, s);
#pragma unroll
            for (int a = 0; a < 3; ++a) n[a] = R.n[a];
        }
        // segmented inclusive sum over runs of equal f (every lane active
        // here), on DPP: within each row of 16 lanes by row shifts, then
        // lane 15 of the previous row to rows 1 and 3, then lane 31 to rows 2
        // and 3, each step taken by the lanes whose run reaches its source
        const int32_t fp = __shfl_up(f, 1, dev::kWave);
        const uint64_t heads = __ballot(lane == 0 || fp != f);
        const uint64_t upto = (2ull << lane) - 1ull;   // lanes 0 .. lane (all 64 at lane 63)
        const int start = 63 - __clzll(heads & upto);
        const int rl = lane & 15;
        // within rows (row_shr:d); once no lane can use a shift, no longer one can
        if (__ballot(rl >= 1 && lane - 1 >= start)) {
            dpp_add<0x111, 0xF>(s, rl >= 1 && lane - 1 >= start);
            if (__ballot(rl >= 2 && lane - 2 >= start)) {
                dpp_add<0x112, 0xF>(s, rl >= 2 && lane - 2 >= start);
                if (__ballot(rl >= 4 && lane - 4 >= start)) {
                    dpp_add<0x114, 0xF>(s, rl >= 4 && lane - 4 >= start);
                    if (__ballot(rl >= 8 && lane - 8 >= start)) dpp_add<0x118, 0xF>(s, rl >= 8 && lane - 8 >= start);
                }
            }
        }
        const bool b15 = (lane & 16) && (lane & ~15) - 1 >= start;   // row_bcast:15 into rows 1 and 3
        if (__ballot(b15)) dpp_add<0x142, 0xA>(s, b15);
        const bool b31 = lane >= 32 && start <= 31;   // row_bcast:31 into rows 2 and 3
        if (__ballot(b31)) dpp_add<0x143, 0xC>(s, b31);
        const bool tail = lane == dev::kWave - 1 || (((heads >> lane) >> 1) & 1ull);
        if (tail && f >= 0) to_lds(f, s, n);
    };

    const int span = nn * Q;
    // Slots are read four per lane (16-byte loads of face ids and weights,
    // 256 slots per wave step; the tile's span starts on a 16-byte boundary
    // as kAdjThreads * Q is a multiple of four), the waves taking every
    // kAdjWaves-th step with the next step's loads in flight; a partial step at
    // the span's end, or rows not 16-byte aligned, go slot by slot.  Live
    // slots are queued in slot order (a lane's at its prefix of the wave's
    // live counts).
    constexpr int kV = kAdjGroup;
    static_assert(kV == 4, "int4 / float4 loads");
    static_assert((kAdjThreads * Q) % kV == 0, "tile spans start on 16-byte boundaries");
    const bool vec = ((reinterpret_cast<uintptr_t>(A.gq) | reinterpret_cast<uintptr_t>(A.face)) & 15u) == 0;
    const int nst = (span + kV * dev::kWave - 1) / (kV * dev::kWave);
    int4 nf;
    float4 nw;
    auto load = [&](int st) {
        const int s0 = st * kV * dev::kWave + kV * lane;
        if (vec && s0 + kV <= span) {
            nf = *reinterpret_cast<const int4 *>(A.face + base + s0);
            nw = *reinterpret_cast<const float4 *>(A.gq + base + s0);
        } else {
            int32_t lf[kV];
            float lw[kV];
#pragma unroll
            for (int k = 0; k < kV; ++k) {
                lf[k] = -1;
                lw[k] = 0.0f;
                if (s0 + k < span) {
                    lf[k] = A.face[base + s0 + k];
                    lw[k] = A.gq[base + s0 + k];
                }
            }
            nf = make_int4(lf[0], lf[1], lf[2], lf[3]);
            nw = make_float4(lw[0], lw[1], lw[2], lw[3]);
        }
    };
    if (wv < nst) load(wv);
    for (int st = wv; st < nst; st += kAdjWaves) {
        const int32_t f[kV] = {nf.x, nf.y, nf.z, nf.w};
        const float w[kV] = {nw.x, nw.y, nw.z, nw.w};
        if (st + kAdjWaves < nst) load(st + kAdjWaves);
        const int s0 = st * kV * dev::kWave + kV * lane;
        int nl = s0 / Q, i = s0 - nl * Q;
        uint32_t meta[kV], live = 0;
#pragma unroll
        for (int k = 0; k < kV; ++k) {
            // false past the span (f = -1)
            live |= (i != 0 && f[k] >= 0 && w[k] != 0.0f) ? 1u << k : 0u;
            meta[k] = ((uint32_t)nl << 5) | (uint32_t)i;
            if (++i == Q) {
                i = 0;
                ++nl;
            }
        }
        const uint32_t cnt = (uint32_t)__popc(live);
        const uint32_t incl = dpp_inclusive_sum(cnt);
        int at = qn + (int)(incl - cnt);
#pragma unroll
        for (int k = 0; k < kV; ++k)
            if ((live >> k) & 1u) {
                qm[at] = meta[k];
                qf[at] = f[k];
                ++at;
            }
        qn += __builtin_amdgcn_readlane((int)incl, dev::kWave - 1);
        while (qn >= dev::kWave) take(qn);
    }
    if (qn > 0) take(qn);
    __syncthreads();

    // the queues are free: vertex table
    for (int i = tid; i < kVHash; i += kAdjThreads) {
        v_key[i] = -1;
#pragma unroll
        for (int a = 0; a < D; ++a) v_acc[i][a] = 0.0f;
    }
    __syncthreads();
    for (int sl = tid; sl < kAdjHash; sl += kAdjThreads) {
        const int32_t f = s_key[sl];
        if (f < 0) continue;
        float v[dev::kRecFloats<D>], n[3];
        dev::load_rec<D>(A.rec, f, v);
        face_normal<D>(v, n);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int32_t vk = A.fidx[(int64_t)f * D + k];
            const float sk = s_acc[sl][k];
            uint32_t h = ((uint32_t)vk * 2654435761u) >> 23;   // 9 bits: kVHash slots
            bool placed = false;
            for (int probe = 0; probe < 32; ++probe) {
                const int32_t prev = atomicCAS(&v_key[h], -1, vk);
                if (prev == -1 || prev == vk) {
#pragma unroll
                    for (int a = 0; a < D; ++a) atomicAdd(&v_acc[h][a], sk * n[a]);
                    placed = true;
                    break;
                }
                h = (h + 1) & (kVHash - 1);
            }
            if (!placed)
#pragma unroll
                for (int a = 0; a < D; ++a) unsafeAtomicAdd(&A.grad[(int64_t)vk * D + a], sk * n[a]);
        }
    }
    __syncthreads();
    for (int i = tid; i < kVHash; i += kAdjThreads) {
        const int32_t vk = v_key[i];
        if (vk < 0) continue;
#pragma unroll
        for (int a = 0; a < D; ++a) unsafeAtomicAdd(&A.grad[(int64_t)vk * D + a], v_acc[i][a]);
    }
    __syncthreads();
}

// Copy c staged node rows (key, q row, face row) from row src to row dst, as
// flat coalesced runs over one wave.
template <int Q>
__device__ __forceinline__ void compact_block(int c, int64_t src, int64_t dst, const uint64_t *__restrict__ skey,
                                              const float *__restrict__ sq, const int32_t *__restrict__ sface,
                                              uint64_t *__restrict__ key, float *__restrict__ q,
                                              int32_t *__restrict__ face) {
    if (c == 0) return;
    for (int r = threadIdx.x; r < c; r += 64) key[dst + r] = skey[src + r];
    const float *__restrict__ qs = sq + src * Q;
    const int32_t *__restrict__ fs = sface + src * Q;
    float *__restrict__ qd = q + dst * Q;
    int32_t *__restrict__ fd = face + dst * Q;
    const int n = c * Q;
    // four loads per array in flight before the stores
    int e = threadIdx.x;
    for (; e + 3 * 64 < n; e += 4 * 64) {
        float a[4];
        int32_t b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = qs[e + u * 64];
            b[u] = fs[e + u * 64];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            qd[e + u * 64] = a[u];
            fd[e + u * 64] = b[u];
        }
    }
    for (; e < n; e += 64) {
        qd[e] = qs[e];
        fd[e] = fs[e];
    }
}


// ---- link fractions, list mode: candidate blocks per face ------------------
// Finest-level block of integer block coordinates c: at level 0 the root's
// linear index; above, the parent's first child (hash table of parent keys,
// linear probing; slot = parent key << 32 | index of its first child, ~0
// empty) plus the child index.  -1: no such block.
struct BlockFind {
    const unsigned long long *hash;
    uint32_t hmask;   // slots - 1
    int hshift;       // 32 - log2(slots)
    int level;
    int R[3];
    const uint32_t *keys;   // the level's sorted keys (a found index is checked against them)
    int64_t n;
};

__device__ __forceinline__ uint32_t hash_slot(uint32_t key, int shift) { return (key * 2654435761u) >> shift; }

template <int D>
__device__ __forceinline__ int64_t find_block(const BlockFind &B, const int c[3]) {
    if (B.level == 0) {
        const int64_t i = ((int64_t)c[2] * B.R[1] + c[1]) * B.R[0] + c[0];
        return i < B.n ? i : -1;
    }
    const int p[3] = {c[0] >> 1, c[1] >> 1, D == 3 ? c[2] >> 1 : 0};
    const uint32_t pk = dev::encode_key<D>(p, B.level - 1, B.R[0], B.R[1]);
    uint32_t ci = (uint32_t)(c[0] & 1) | ((uint32_t)(c[1] & 1) << 1);
    if (D == 3) ci |= (uint32_t)(c[2] & 1) << 2;
    uint32_t s = hash_slot(pk, B.hshift);
    for (uint32_t probe = 0; probe <= B.hmask; ++probe) {
        const unsigned long long v = B.hash[s];
        if (v == ~0ull) return -1;
        if ((uint32_t)(v >> 32) == pk) {
            const int64_t i = (int64_t)(uint32_t)v + ci;
            return i < B.n && B.keys[i] == ((pk << D) | ci) ? i : -1;
        }
        s = (s + 1) & B.hmask;
    }
    return -1;
}

// Block i of the level: its node mask zeroed and, above level 0, the parent
// of every first child (child index 0) inserted into the table.
template <int D>
__device__ __forceinline__ void link_block_item(const uint32_t *keys, int64_t i, unsigned long long *hash,
                                                uint32_t hmask, int hshift, unsigned long long *mask) {
    mask[i] = 0ull;
    if (!hash) return;
    const uint32_t key = keys[i];
    if (key & ((1u << D) - 1u)) return;
    const uint32_t pk = key >> D;
    const unsigned long long v = ((unsigned long long)pk << 32) | (uint32_t)i;
    uint32_t s = hash_slot(pk, hshift);
    for (uint32_t probe = 0; probe <= hmask; ++probe) {
        if (atomicCAS(&hash[s], ~0ull, v) == ~0ull) break;
        s = (s + 1) & hmask;
    }
}

// Block ranges of a face's candidate blocks, per axis in FP64: block b is a
// candidate when its link box [lo + (4b - 0.5) dx - eps, lo + (4b + 4.5) dx +
// eps] (FP32 in the link kernels) meets the face box widened by m = 2 eps,
// a margin above the FP32 rounding of those bounds, so the list holds every
// face the kernels' own FP32 box test keeps (and a few more, which it drops).
struct LinkFaceGrid {
    double lo[3], dx[3], m[3];
    int NB[3];
};

// One wave per kLinkFaceG faces: count (kScatter false) or write (true) each
// face into the list of every existing candidate block.  The (face, block
// position) pairs of the wave's faces are taken 64 at a time, one per lane,
// so the hash probes of many pairs are in flight together.  A face with more
// than max_coords candidate positions is skipped by both passes (the bound
// the list was sized with makes that impossible for the geometry it was
// measured on; the test keeps the writes inside the list whatever happens, and
// `over`, when given, records the skip), and so is a write at or past cap.
constexpr int kLinkFaceG = 16;

template <int D, bool kScatter>
__device__ __forceinline__ void link_faces_wave(const float *aabb, int64_t F, const LinkFaceGrid &G,
                                                const BlockFind &B, int64_t max_coords, uint32_t *cnt,
                                                const uint32_t *loff, uint32_t *cursor, int32_t *list, uint32_t *lblk,
                                                uint32_t cap, int64_t f0, uint32_t *over = nullptr) {
    __shared__ int s_i[kLinkFaceG][8];   // per face: first block per axis, positions per axis, pair prefix
    const int lane = dev::lane_id();
    uint32_t npos = 0;
    if (lane < kLinkFaceG) {
        const int64_t f = f0 + lane;
        int b0[3] = {0, 0, 0}, nb[3] = {1, 1, 1};
        bool any = f < F;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (!any) break;
            const double mn = aabb[(int64_t)a * F + f], mx = aabb[(int64_t)(D + a) * F + f];
            double l = ceil((mn - G.lo[a] - G.m[a] - 4.5 * G.dx[a]) / (4.0 * G.dx[a]));
            double h = floor((mx - G.lo[a] + G.m[a] + 0.5 * G.dx[a]) / (4.0 * G.dx[a]));
            l = l < 0.0 ? 0.0 : l;
            h = h > (double)(G.NB[a] - 1) ? (double)(G.NB[a] - 1) : h;
            if (!(l <= h)) {   // outside the grid, or a non-finite coordinate
                any = false;
                break;
            }
            b0[a] = (int)l;
            nb[a] = (int)(h - l) + 1;
        }
        if (any && (int64_t)nb[0] * nb[1] * nb[2] <= max_coords) npos = (uint32_t)(nb[0] * nb[1] * nb[2]);
        else if (any && over) atomicOr(over, 8u);   // beyond the bound the lists were sized with
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            s_i[lane][a] = b0[a];
            s_i[lane][3 + a] = nb[a];
        }
    }
    const uint32_t incl = dev::wave_inclusive_sum(npos);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, dev::kWave - 1);
    if (lane < kLinkFaceG) s_i[lane][6] = (int)(incl - npos);
    dev::wave_sync();
    for (uint32_t c0 = 0; c0 < total; c0 += dev::kWave) {
        const uint32_t v = c0 + (uint32_t)lane;
        if (v >= total) break;
        int k = 0;   // the last face whose pairs start at or before v
#pragma unroll
        for (int step = kLinkFaceG / 2; step >= 1; step >>= 1)
            if ((uint32_t)s_i[k + step][6] <= v) k += step;
        uint32_t u = v - (uint32_t)s_i[k][6];
        int c[3];
        c[0] = s_i[k][0] + (int)(u % (uint32_t)s_i[k][3]);
        u /= (uint32_t)s_i[k][3];
        c[1] = s_i[k][1] + (int)(u % (uint32_t)s_i[k][4]);
        c[2] = s_i[k][2] + (int)(u / (uint32_t)s_i[k][4]);
        const int64_t idx = find_block<D>(B, c);
        if (idx < 0) continue;
        if constexpr (kScatter) {
            const uint32_t pos = loff[idx] + atomicAdd(&cursor[idx], 1u);
            if (pos < cap) {
                list[pos] = (int32_t)(f0 + k);
                lblk[pos] = (uint32_t)idx;
            }
        } else {
            atomicAdd(&cnt[idx], 1u);
        }
    }
}

// Nodes of blocks b0 .. b0 + 63 (below n; b0 wave-uniform): every lane loads
// one block's mask, first node index and key, then the wave writes the
// blocks' nodes block by block, lane i writing cell i when it is set at
// noff + (set cells below i), so each block's nodes go out as one coalesced
// run of keys and block indices.
template <int D>
__device__ __forceinline__ void node_map_chunk(const unsigned long long *mask, const uint32_t *noff,
                                               const uint32_t *keys, int64_t b0, int64_t n, uint32_t *nblk,
                                               uint64_t *node_key) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    const int lane = dev::lane_id();
    const int64_t b = b0 + lane;
    unsigned long long m = 0ull;
    uint32_t off = 0, key = 0;
    if (b < n) {
        m = mask[b];
        off = noff[b];
        key = keys[b];
    }
    for (uint64_t live = __ballot(m != 0ull); live; live &= live - 1ull) {
        const int j = __builtin_ctzll(live);
        const unsigned long long mj = ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(m >> 32), j) << 32) |
                                      (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)m, j);
        const uint32_t oj = (uint32_t)__builtin_amdgcn_readlane((int)off, j);
        const uint32_t kj = (uint32_t)__builtin_amdgcn_readlane((int)key, j);
        if (lane < CELLS && ((mj >> lane) & 1ull)) {
            const int64_t k = (int64_t)oj + dev::lanes_below(mj);
            nblk[k] = (uint32_t)(b0 + j);
            node_key[k] = (uint64_t)kj * CELLS + (uint64_t)lane;
        }
    }
}

}  // namespace kern
}  // namespace agal
