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
#include "kernels.hpp"

namespace agal {

namespace {

using namespace kern;

#define AGAL_GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

template <int D>
__global__ void k_bin_count(const float *aabb, int64_t F, dev::BinGrid g, uint32_t *count) {
    AGAL_GRID_STRIDE(f, F) bin_count_item<D>(aabb, F, g, count, f);
}

template <int D>
__global__ void k_bin_scatter(const float *aabb, int64_t F, dev::BinGrid g, const uint32_t *off, uint32_t *cursor,
                              int32_t *ids) {
    AGAL_GRID_STRIDE(f, F) bin_scatter_item<D>(aabb, F, g, off, cursor, ids, f);
}

__global__ __launch_bounds__(64) void k_bin_canon_small(int32_t *ids, const uint32_t *off, int64_t nb,
                                                        uint32_t *big_list, uint32_t *big_count) {
    bin_canon_group(ids, off, nb, (int64_t)blockIdx.x * dev::kWave, big_list, big_count, 0u);
}

template <int D>
__global__ __launch_bounds__(kBigThreads) void k_bin_canon_big(const float *aabb, int64_t F, dev::BinGrid g,
                                                               const uint32_t *off, int32_t *ids,
                                                               const uint32_t *big_list, const uint32_t *big_count) {
    const uint32_t nbig = *big_count;
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) bin_canon_big_bin<D>(aabb, F, g, off, ids, big_list[bi]);
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
    // one zeroed work buffer: per-bin counts, per-bin scatter cursors, the
    // oversized-bin counter, and the scan's look-back status words
    const int64_t tiles = scan_tiles(nb);
    const int64_t work_words = 2 * nb + 2 + 2 * (tiles + 1);
    uint32_t *work = nullptr;
    agal_status st = dev_alloc(ctx->mem, &work, (size_t)work_words, s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &bn->off, (size_t)nb + 1, s);
    if (st != AGAL_OK) {
        dev_free(ctx->mem, work, s);
        agal_destroy_bins(bn);
        return st;
    }
    fill_u32(work, 0u, work_words, s);
    uint32_t *count = work;
    uint32_t *cursor = work + nb;
    uint32_t *big_count = work + 2 * nb;
    uint64_t *scan_status = reinterpret_cast<uint64_t *>(work + ((2 * nb + 3) & ~int64_t(1)));
    {
    ProfScope prof(ctx, "bin_count", s);
    if (D == 3)
        hipLaunchKernelGGL(k_bin_count<3>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, grid, count);
    else
        hipLaunchKernelGGL(k_bin_count<2>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, grid, count);
    }
    uint32_t P = 0;
    st = scan_u32_total(ctx, count, bn->off, nb, scan_status, &P, s);
    bn->P = P;
    uint32_t *big = nullptr;   // the oversized bins (big_count[0] of them)
    const int64_t big_cap = (int64_t)P / kCanonCap + 1;
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &bn->ids, (size_t)std::max<uint32_t>(P, 1u), s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &big, (size_t)big_cap, s);
    if (st != AGAL_OK) {
        dev_free(ctx->mem, work, s);
        dev_free(ctx->mem, big, s);
        agal_destroy_bins(bn);
        return st;
    }
    {
    ProfScope prof(ctx, "bin_scatter", s);
    if (D == 3)
        hipLaunchKernelGGL(k_bin_scatter<3>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, grid, bn->off,
                           cursor, bn->ids);
    else
        hipLaunchKernelGGL(k_bin_scatter<2>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, grid, bn->off,
                           cursor, bn->ids);
    }
    const int64_t groups = (nb + dev::kWave - 1) / dev::kWave;
    {
    ProfScope prof(ctx, "bin_canon", s);
    hipLaunchKernelGGL(k_bin_canon_small, dim3((unsigned)groups), dim3(dev::kWave), 0, s, bn->ids, bn->off, nb,
                       big, big_count);
    }
    const unsigned big_grid = (unsigned)std::min<int64_t>(big_cap, 256);
    {
    ProfScope prof(ctx, "bin_canon_big", s);
    if (D == 3)
        hipLaunchKernelGGL(k_bin_canon_big<3>, dim3(big_grid), dim3(kBigThreads), 0, s, g->aabb, g->F, grid, bn->off,
                           bn->ids, big, big_count);
    else
        hipLaunchKernelGGL(k_bin_canon_big<2>, dim3(big_grid), dim3(kBigThreads), 0, s, g->aabb, g->F, grid, bn->off,
                           bn->ids, big, big_count);
    }
    dev_free(ctx->mem, work, s);
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
