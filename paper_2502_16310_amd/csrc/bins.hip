// Spatial binning (paper Sec. II-C-3): faces are distributed to a uniform grid
// of B^D bins over [lo, hi].  Output is the three-array form the paper
// describes (ids grouped by bin, per-bin counts as offset differences, first
// index per bin) as a CSR with ascending face ids inside each bin.
//
// Kernels: count (one thread per face, atomics per touched bin) -> exclusive
// scan -> scatter (atomic cursors) -> canonical order (each bin's segment
// sorted by rank in LDS; bins too large for LDS are rebuilt by an ordered
// sweep over all faces, which only happens when B is tiny).
#include <algorithm>

#include "agal_internal.hpp"
#include "device.hpp"

namespace agal {

namespace {

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

template <int D>
__global__ void k_bin_count(const float *aabb, int64_t F, dev::BinGrid g, uint32_t *count) {
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
        int lo[3], hi[3];
        face_bin_range<D>(aabb, F, f, g, lo, hi);
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x)
                    atomicAdd(&count[((int64_t)z * g.B + y) * g.B + x], 1u);
    }
}

template <int D>
__global__ void k_bin_scatter(const float *aabb, int64_t F, dev::BinGrid g, const uint32_t *off, uint32_t *cursor,
                              int32_t *ids) {
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
        int lo[3], hi[3];
        face_bin_range<D>(aabb, F, f, g, lo, hi);
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    int64_t b = ((int64_t)z * g.B + y) * g.B + x;
                    uint32_t pos = off[b] + atomicAdd(&cursor[b], 1u);
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

// One wave per group of 64 consecutive bins.
__global__ __launch_bounds__(64) void k_bin_canon_small(int32_t *ids, const uint32_t *off, int64_t nb,
                                                        uint32_t *big_list, uint32_t *big_count) {
    __shared__ uint32_t s_off[dev::kWave + 1];
    __shared__ int32_t s_val[kCanonCap];
    const int64_t b0 = (int64_t)blockIdx.x * dev::kWave;
    const int nbins = (int)std::min<int64_t>(dev::kWave, nb - b0);
    const int lane = threadIdx.x;
    for (int i = lane; i <= nbins; i += dev::kWave) s_off[i] = off[b0 + i];
    __syncthreads();
    const uint32_t g0 = s_off[0], g1 = s_off[nbins];
    if (g1 - g0 <= 1) return;
    if (g1 - g0 <= (uint32_t)kCanonCap) {
        rank_sort_segment(ids, s_off, nbins, g0, g1, s_val);
        return;
    }
    // group too large: bin by bin
    for (int b = 0; b < nbins; ++b) {
        const uint32_t a0 = s_off[b], a1 = s_off[b + 1];
        if (a1 - a0 <= 1) continue;
        if (a1 - a0 <= (uint32_t)kCanonCap) {
            __shared__ uint32_t s_one[2];
            if (lane == 0) { s_one[0] = a0; s_one[1] = a1; }
            __syncthreads();
            rank_sort_segment(ids, s_one, 1, a0, a1, s_val);
        } else if (lane == 0) {
            uint32_t k = atomicAdd(big_count, 1u);
            big_list[k] = (uint32_t)(b0 + b);
        }
    }
}

// Bins with more than kCanonCap ids: rewrite the segment by an ordered sweep
// over all faces (membership recomputed from the bounding boxes).
template <int D>
__global__ __launch_bounds__(kBigThreads) void k_bin_canon_big(const float *aabb, int64_t F, dev::BinGrid g,
                                                               const uint32_t *off, int32_t *ids,
                                                               const uint32_t *big_list, const uint32_t *big_count) {
    __shared__ uint32_t s_wsum[kBigThreads / dev::kWave];
    const uint32_t nbig = *big_count;
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x % dev::kWave;
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const int64_t b = big_list[bi];
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

unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 8192) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

}  // namespace agal

using namespace agal;

extern "C" {

agal_status agal_bin_faces(agal_geom g, const float lo[3], const float hi[3], int32_t B, void *stream, agal_bins *out) {
    if (!g || !lo || !hi || !out) return fail(AGAL_EINVAL, "agal_bin_faces: NULL argument");
    if (B < 1) return fail(AGAL_EINVAL, "agal_bin_faces: B must be >= 1 (got %d)", B);
    const int D = g->dim;
    int64_t nb = 1;
    for (int a = 0; a < D; ++a) {
        if (!(hi[a] > lo[a])) return fail(AGAL_EINVAL, "agal_bin_faces: hi must exceed lo on every axis");
        if (nb > ((int64_t)1 << 31) / B) return fail(AGAL_EINVAL, "agal_bin_faces: B^D exceeds 2^31");
        nb *= B;
    }
    hipStream_t s = (hipStream_t)stream;
    agal_context ctx = g->ctx;

    auto *bn = new (std::nothrow) agal_bins_t();
    if (!bn) return fail(AGAL_ENOMEM, "agal_bin_faces: host allocation failed");
    bn->ctx = ctx;
    bn->geom_id = g->id;
    bn->stream = s;
    bn->dim = D;
    bn->B = B;
    bn->nb = nb;
    dev::BinGrid grid{};
    grid.B = B;
    for (int a = 0; a < 3; ++a) {
        bn->lo[a] = a < D ? lo[a] : 0.0f;
        bn->hi[a] = a < D ? hi[a] : 1.0f;
        bn->s[a] = (float)B / (bn->hi[a] - bn->lo[a]);
        grid.lo[a] = bn->lo[a];
        grid.s[a] = bn->s[a];
    }
    uint32_t *count = nullptr;
    agal_status st = dev_alloc(ctx->mem, &count, (size_t)nb, s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &bn->off, (size_t)nb + 1, s);
    if (st != AGAL_OK) {
        dev_free(ctx->mem, count, s);
        agal_destroy_bins(bn);
        return st;
    }
    fill_u32(count, 0u, nb, s);
    {
    ProfScope prof(ctx, "bin_count", s);
    if (D == 3)
        hipLaunchKernelGGL(k_bin_count<3>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, grid, count);
    else
        hipLaunchKernelGGL(k_bin_count<2>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, grid, count);
    }
    st = scan_u32(ctx, count, bn->off, nb, s);
    uint32_t P = 0;
    if (st == AGAL_OK) {
        const uint32_t *src[1] = {bn->off + nb};
        st = read_back_u32(ctx, src, 1, &P, s);
    }
    bn->P = P;
    uint32_t *big = nullptr;
    const int64_t big_cap = (int64_t)P / kCanonCap + 2;
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &bn->ids, (size_t)std::max<uint32_t>(P, 1u), s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &big, (size_t)big_cap, s);
    if (st != AGAL_OK) {
        dev_free(ctx->mem, count, s);
        dev_free(ctx->mem, big, s);
        agal_destroy_bins(bn);
        return st;
    }
    fill_u32(count, 0u, nb, s);   // reused as scatter cursors
    fill_u32(big, 0u, 1, s);      // big[0] = number of oversized bins; list follows
    {
    ProfScope prof(ctx, "bin_scatter", s);
    if (D == 3)
        hipLaunchKernelGGL(k_bin_scatter<3>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, grid, bn->off,
                           count, bn->ids);
    else
        hipLaunchKernelGGL(k_bin_scatter<2>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, grid, bn->off,
                           count, bn->ids);
    }
    const int64_t groups = (nb + dev::kWave - 1) / dev::kWave;
    {
    ProfScope prof(ctx, "bin_canon", s);
    hipLaunchKernelGGL(k_bin_canon_small, dim3((unsigned)groups), dim3(dev::kWave), 0, s, bn->ids, bn->off, nb,
                       big + 1, big);
    }
    const unsigned big_grid = (unsigned)std::min<int64_t>(big_cap, 256);
    {
    ProfScope prof(ctx, "bin_canon_big", s);
    if (D == 3)
        hipLaunchKernelGGL(k_bin_canon_big<3>, dim3(big_grid), dim3(kBigThreads), 0, s, g->aabb, g->F, grid, bn->off,
                           bn->ids, big + 1, big);
    else
        hipLaunchKernelGGL(k_bin_canon_big<2>, dim3(big_grid), dim3(kBigThreads), 0, s, g->aabb, g->F, grid, bn->off,
                           bn->ids, big + 1, big);
    }
    dev_free(ctx->mem, count, s);
    dev_free(ctx->mem, big, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        agal_destroy_bins(bn);
        return fail(AGAL_EHIP, "agal_bin_faces: launch failed: %s", hipGetErrorString(e));
    }
    *out = bn;
    return AGAL_OK;
}

agal_status agal_bins_view(agal_bins b, const uint32_t **d_offsets, const int32_t **d_face_ids, int64_t *n_bins,
                           int64_t *n_entries) {
    if (!b) return fail(AGAL_EINVAL, "agal_bins_view: NULL bins");
    if (d_offsets) *d_offsets = b->off;
    if (d_face_ids) *d_face_ids = b->ids;
    if (n_bins) *n_bins = b->nb;
    if (n_entries) *n_entries = b->P;
    return AGAL_OK;
}

void agal_destroy_bins(agal_bins b) {
    if (!b) return;
    dev_free(b->ctx->mem, b->off, b->stream);
    dev_free(b->ctx->mem, b->ids, b->stream);
    delete b;
}

}  // extern "C"
