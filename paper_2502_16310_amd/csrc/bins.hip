// Spatial binning (paper Sec. II-C-3): faces are distributed to a uniform grid
// of B^D bins over [lo, hi].  Output is the three-array form the paper
// describes (ids grouped by bin, per-bin counts as offset differences, first
// index per bin) as a CSR with ascending face ids inside each bin.
//
// Kernels: count (one thread per face, atomics per touched bin) -> exclusive
// scan -> scatter (atomic cursors) -> canonical order (each bin's segment
// sorted by rank in LDS: a group of 64 bins at once when its ids fit, else a
// workgroup per bin; bins too large for LDS are rebuilt by an ordered sweep
// over all faces, which only happens when B is tiny).
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
                                                        uint32_t *med_list, uint32_t *big_list, uint32_t *counts) {
    bin_canon_group(ids, off, nb, (int64_t)blockIdx.x * dev::kWave, med_list, big_list, counts, 0u);
}

__global__ __launch_bounds__(kMedThreads) void k_bin_canon_medium(int32_t *ids, const uint32_t *off,
                                                                  const uint32_t *med_list, const uint32_t *counts) {
    const uint32_t nmed = counts[0];
    for (uint32_t i = blockIdx.x; i < nmed; i += gridDim.x) bin_canon_medium(ids, off, med_list[i]);
}

template <int D>
__global__ __launch_bounds__(kBigThreads) void k_bin_canon_big(const float *aabb, int64_t F, dev::BinGrid g,
                                                               const uint32_t *off, int32_t *ids,
                                                               const uint32_t *big_list, const uint32_t *big_count /* counts */) {
    const uint32_t nbig = big_count[1];
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) bin_canon_big_bin<D>(aabb, F, g, off, ids, big_list[bi]);
}

unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 8192) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// Validated bin grid of a call: B bins per axis over [lo, hi].
struct GridSpec {
    dev::BinGrid grid{};
    float lo[3], hi[3], s[3];
    int64_t nb = 1;
};

agal_status grid_spec(const char *what, int D, const float lo[3], const float hi[3], int32_t B, GridSpec *out) {
    if (B < 1) return fail(AGAL_EINVAL, "%s: B must be >= 1 (got %d)", what, B);
    int64_t nb = 1;
    for (int a = 0; a < D; ++a) {
        if (!(hi[a] > lo[a])) return fail(AGAL_EINVAL, "%s: hi must exceed lo on every axis", what);
        if (nb > ((int64_t)1 << 31) / B) return fail(AGAL_EINVAL, "%s: B^D exceeds 2^31", what);
        nb *= B;
    }
    out->nb = nb;
    out->grid.B = B;
    for (int a = 0; a < 3; ++a) {
        out->lo[a] = a < D ? lo[a] : 0.0f;
        out->hi[a] = a < D ? hi[a] : 1.0f;
        out->s[a] = (float)B / (out->hi[a] - out->lo[a]);
        out->grid.lo[a] = out->lo[a];
        out->grid.s[a] = out->s[a];
    }
    return AGAL_OK;
}

// Work words of one binning call over nb bins: per-bin counts, per-bin
// scatter cursors, the medium- and big-bin list counters, then the scan's
// look-back status words (64-bit).  All start at zero.
int64_t bin_work_words(int64_t nb) { return 2 * nb + 2 + 2 * (scan_tiles(nb) + 1); }

struct BinWork {
    uint32_t *count, *cursor, *lists;   // lists[0], lists[1]: medium and big bin counts
    uint64_t *scan_status;
};

BinWork bin_work(uint32_t *work, int64_t nb) {
    return BinWork{work, work + nb, work + 2 * nb, reinterpret_cast<uint64_t *>(work + ((2 * nb + 3) & ~int64_t(1)))};
}

// Count pass and scan: zeroes `work`, fills off[0..nb] and returns the entry
// total P (the one host wait).  ctx_timed: the context whose kernel timing
// records the launches, or null for none.
agal_status bin_count_scan(agal_context ctx, agal_context ctx_timed, agal_geom g, const GridSpec &gs, uint32_t *work,
                           uint32_t *off, uint32_t *P, hipStream_t s) {
    const int64_t nb = gs.nb;
    fill_u32(work, 0u, bin_work_words(nb), s);
    const BinWork w = bin_work(work, nb);
    {
        ProfScope prof(ctx_timed, "bin_count", s);
        if (g->dim == 3)
            hipLaunchKernelGGL(k_bin_count<3>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, gs.grid, w.count);
        else
            hipLaunchKernelGGL(k_bin_count<2>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, gs.grid, w.count);
    }
    AGAL_TRY_HIP(hipGetLastError());
    return scan_u32_total(ctx, w.count, off, nb, w.scan_status, P, s, ctx_timed != nullptr);
}

// Scatter and canonical order into ids[0..P) (offsets from bin_count_scan);
// med: room for nb bin indices, big: for P / kCanonCap + 1.
agal_status bin_scatter_canon(agal_context ctx_timed, agal_geom g, const GridSpec &gs, uint32_t *work,
                              const uint32_t *off, int32_t *ids, uint32_t P, uint32_t *med, uint32_t *big,
                              hipStream_t s) {
    const int64_t nb = gs.nb;
    const BinWork w = bin_work(work, nb);
    {
        ProfScope prof(ctx_timed, "bin_scatter", s);
        if (g->dim == 3)
            hipLaunchKernelGGL(k_bin_scatter<3>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, gs.grid, off,
                               w.cursor, ids);
        else
            hipLaunchKernelGGL(k_bin_scatter<2>, dim3(grid_for(g->F)), dim3(256), 0, s, g->aabb, g->F, gs.grid, off,
                               w.cursor, ids);
    }
    const int64_t groups = (nb + dev::kWave - 1) / dev::kWave;
    {
        ProfScope prof(ctx_timed, "bin_canon", s);
        hipLaunchKernelGGL(k_bin_canon_small, dim3((unsigned)groups), dim3(dev::kWave), 0, s, ids, off, nb, med, big,
                           w.lists);
        hipLaunchKernelGGL(k_bin_canon_medium, dim3((unsigned)std::min<int64_t>(nb, 8192)), dim3(kMedThreads), 0, s,
                           ids, off, med, w.lists);
    }
    const unsigned big_grid = (unsigned)std::min<int64_t>((int64_t)P / kCanonCap + 1, 256);
    {
        ProfScope prof(ctx_timed, "bin_canon_big", s);
        if (g->dim == 3)
            hipLaunchKernelGGL(k_bin_canon_big<3>, dim3(big_grid), dim3(kBigThreads), 0, s, g->aabb, g->F, gs.grid,
                               off, ids, big, w.lists);
        else
            hipLaunchKernelGGL(k_bin_canon_big<2>, dim3(big_grid), dim3(kBigThreads), 0, s, g->aabb, g->F, gs.grid,
                               off, ids, big, w.lists);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(AGAL_EHIP, "binning: launch failed: %s", hipGetErrorString(e));
    return AGAL_OK;
}

// Scratch of agal_bin_faces_noalloc: a file-scope device array (each device
// holds its own copy for the life of the process).  Host code never passes
// the array's name to a kernel: on the host it is only a stand-in, and its
// device address comes from hipGetSymbolAddress, taken once per device when a
// context is created there.
constexpr int64_t kNoallocScratchWords = (int64_t(32) << 20) / 4;   // 32 MiB
static __device__ __align__(256) uint32_t scratch[kNoallocScratchWords];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch[kMaxDevices] = {};

}  // namespace

agal_status bin_scratch_resolve(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(AGAL_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return AGAL_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(AGAL_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    }
    g_scratch[device] = static_cast<uint32_t *>(p);
    return AGAL_OK;
}

}  // namespace agal

using namespace agal;

extern "C" {

agal_status agal_bin_faces(agal_geom g, const float lo[3], const float hi[3], int32_t B, void *stream, agal_bins *out) {
    if (!g || !lo || !hi || !out) return fail(AGAL_EINVAL, "agal_bin_faces: NULL argument");
    GridSpec gs;
    AGAL_TRY(grid_spec("agal_bin_faces", g->dim, lo, hi, B, &gs));
    const int64_t nb = gs.nb;
    hipStream_t s = (hipStream_t)stream;
    agal_context ctx = g->ctx;

    auto *bn = new (std::nothrow) agal_bins_t();
    if (!bn) return fail(AGAL_ENOMEM, "agal_bin_faces: host allocation failed");
    bn->ctx = ctx;
    bn->geom_id = g->id;
    bn->stream = s;
    bn->dim = g->dim;
    bn->B = B;
    bn->nb = nb;
    for (int a = 0; a < 3; ++a) {
        bn->lo[a] = gs.lo[a];
        bn->hi[a] = gs.hi[a];
        bn->s[a] = gs.s[a];
    }
    uint32_t *work = nullptr, *med = nullptr, *big = nullptr;
    auto cleanup = [&](agal_status st) {
        dev_free(ctx->mem, work, s);
        dev_free(ctx->mem, med, s);
        dev_free(ctx->mem, big, s);
        if (st != AGAL_OK) agal_destroy_bins(bn);
        return st;
    };
    agal_status st = dev_alloc(ctx->mem, &work, (size_t)bin_work_words(nb), s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &bn->off, (size_t)nb + 1, s);
    uint32_t P = 0;
    if (st == AGAL_OK) st = bin_count_scan(ctx, ctx, g, gs, work, bn->off, &P, s);
    if (st != AGAL_OK) return cleanup(st);
    bn->P = P;
    st = dev_alloc(ctx->mem, &bn->ids, (size_t)std::max<uint32_t>(P, 1u), s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &med, (size_t)nb, s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &big, (size_t)P / kCanonCap + 1, s);
    if (st == AGAL_OK) st = bin_scatter_canon(ctx, g, gs, work, bn->off, bn->ids, P, med, big, s);
    if (cleanup(st) != AGAL_OK) return st;
    *out = bn;
    return AGAL_OK;
}

agal_status agal_bin_faces_noalloc(agal_geom g, const float lo[3], const float hi[3], int32_t B, uint32_t *d_offsets,
                                   int32_t *d_face_ids, int64_t ids_capacity, void *stream, int64_t *n_entries) {
    if (!g || !lo || !hi || !d_offsets || !n_entries || (ids_capacity > 0 && !d_face_ids))
        return fail(AGAL_EINVAL, "agal_bin_faces_noalloc: NULL argument");
    if (ids_capacity < 0) return fail(AGAL_EINVAL, "agal_bin_faces_noalloc: negative ids_capacity");
    GridSpec gs;
    AGAL_TRY(grid_spec("agal_bin_faces_noalloc", g->dim, lo, hi, B, &gs));
    agal_context ctx = g->ctx;
    const int dev_id = ctx->device;
    uint32_t *base = nullptr;
    if (dev_id >= 0 && dev_id < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch[dev_id];
    }
    if (!base)
        return fail(AGAL_EHIP, "agal_bin_faces_noalloc: the scratch address of device %d is unknown (%s)", dev_id,
                    "hipGetSymbolAddress failed when the context was created");
    // scratch: the work words, the medium-bin list (one word per bin), then
    // the big-bin list (at most ids_capacity / kCanonCap + 1 bins hold more
    // than kCanonCap ids)
    const int64_t work_words = bin_work_words(gs.nb);
    const int64_t big_words = std::min<int64_t>(ids_capacity, (int64_t)UINT32_MAX) / kCanonCap + 1;
    if (work_words + gs.nb + big_words > kNoallocScratchWords)
        return fail(AGAL_EINVAL,
                    "agal_bin_faces_noalloc: %lld bins and %lld id slots need %lld scratch words; the fixed scratch "
                    "holds %lld (at most about %lld bins)",
                    (long long)gs.nb, (long long)ids_capacity, (long long)(work_words + gs.nb + big_words),
                    (long long)kNoallocScratchWords, (long long)((kNoallocScratchWords - big_words) / 3 - 2048));
    hipStream_t s = (hipStream_t)stream;
    uint32_t P = 0;
    AGAL_TRY(bin_count_scan(ctx, nullptr, g, gs, base, d_offsets, &P, s));
    *n_entries = P;
    if ((int64_t)P > ids_capacity)
        return fail(AGAL_ECAPACITY, "agal_bin_faces_noalloc: %u (face, bin) entries exceed ids_capacity %lld", P,
                    (long long)ids_capacity);
    return bin_scatter_canon(nullptr, g, gs, base, d_offsets, d_face_ids, P, base + work_words,
                             base + work_words + gs.nb, s);
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
