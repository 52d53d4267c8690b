// Re-adaptation bookkeeping for a moving body.  The paper refines once,
// before the solver, and names moving geometry as the case where the cost of
// rebuilding the bins every step decides the bin density (Results
// discussion); refinement and coarsening of the blocks themselves come from
// the forest-of-octrees scheme it builds on (Sec. II-C-1).  Here a step of a
// moving body is: import the moved faces, bin them, refine from the roots (the
// re-adapted forest is the near-wall forest of the new geometry), then relate
// the new forest to the previous one level by level, which is what a solver
// needs to carry its data over: per new block its index in the old level (or
// none) and whether it was kept, created, refined (a leaf that gained
// children) or coarsened (children removed); per old block whether it was
// removed.
//
// Both key lists of a level are sorted, so every lookup is a binary search;
// the 64 lanes of a wave look up 64 consecutive keys, whose search paths
// share their upper levels in the cache.  Counts per level and state are
// reduced per workgroup and added once per workgroup.
#include <algorithm>
#include <cstring>

#include "agal_internal.hpp"
#include "device.hpp"

struct agal_forest_diff_t {
    agal_context ctx = nullptr;
    hipStream_t stream = nullptr;
    int L = 0;
    int64_t n_new[agal::kMaxLevels + 1] = {};
    int64_t n_old[agal::kMaxLevels + 1] = {};
    int32_t *old_index[agal::kMaxLevels + 1] = {};
    uint8_t *state[agal::kMaxLevels + 1] = {};
    uint8_t *removed[agal::kMaxLevels + 1] = {};
    unsigned long long counts[agal::kMaxLevels + 1][4] = {};   // created, refined, coarsened, removed
};

namespace agal {
namespace {

constexpr int kDiffThreads = 256;

__device__ __forceinline__ int64_t find_key(const uint32_t *keys, int64_t n, uint32_t k) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const uint32_t v = keys[mid];
        if (v == k) return mid;
        if (v < k) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// New blocks of one level: old index, state, and the created / refined /
// coarsened counts.
__global__ __launch_bounds__(kDiffThreads) void k_diff_new(const uint32_t *nkeys, const uint8_t *nleaf, int64_t nn,
                                                           const uint32_t *okeys, const uint8_t *oleaf, int64_t no,
                                                           int32_t *old_index, uint8_t *state,
                                                           unsigned long long *counts) {
    __shared__ uint32_t s_acc[3];
    uint32_t c[3] = {0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * kDiffThreads + threadIdx.x; i < nn;
         i += (int64_t)gridDim.x * kDiffThreads) {
        const int64_t j = find_key(okeys, no, nkeys[i]);
        uint8_t st = 0;
        if (j < 0) st = 1;
        else if (oleaf[j] && !nleaf[i]) st = 2;
        else if (!oleaf[j] && nleaf[i]) st = 3;
        old_index[i] = (int32_t)j;
        state[i] = st;
        if (st) ++c[st - 1];
    }
    if (threadIdx.x < 3) s_acc[threadIdx.x] = 0u;
    __syncthreads();
    const int lane = dev::lane_id();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // wave sums by shuffles, one LDS atomic per wave
        uint32_t v = c[k];
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, dev::kWave);
        if (lane == 0 && v) atomicAdd(&s_acc[k], v);
    }
    __syncthreads();
    if (threadIdx.x < 3 && s_acc[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)s_acc[threadIdx.x]);
}

// Old blocks of one level: removed flag and count.
__global__ __launch_bounds__(kDiffThreads) void k_diff_old(const uint32_t *okeys, int64_t no, const uint32_t *nkeys,
                                                           int64_t nn, uint8_t *removed, unsigned long long *count) {
    __shared__ uint32_t s_acc;
    uint32_t c = 0u;
    for (int64_t j = (int64_t)blockIdx.x * kDiffThreads + threadIdx.x; j < no;
         j += (int64_t)gridDim.x * kDiffThreads) {
        const bool gone = find_key(nkeys, nn, okeys[j]) < 0;
        removed[j] = gone ? 1 : 0;
        c += gone ? 1u : 0u;
    }
    if (threadIdx.x == 0) s_acc = 0u;
    __syncthreads();
    uint32_t v = c;
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, dev::kWave);
    if (dev::lane_id() == 0 && v) atomicAdd(&s_acc, v);
    __syncthreads();
    if (threadIdx.x == 0 && s_acc) atomicAdd(count, (unsigned long long)s_acc);
}

bool same_grid(agal_forest a, agal_forest b) {
    if (a->dim != b->dim || a->L != b->L) return false;
    for (int k = 0; k < 3; ++k)
        if (a->roots[k] != b->roots[k] || std::memcmp(&a->lo[k], &b->lo[k], 4) || std::memcmp(&a->hi[k], &b->hi[k], 4))
            return false;
    return true;
}

}  // namespace
}  // namespace agal

using namespace agal;

extern "C" {

agal_status agal_forest_diff_create(agal_forest old_f, agal_forest new_f, void *stream, agal_forest_diff *out) {
    if (!old_f || !new_f || !out) return fail(AGAL_EINVAL, "agal_forest_diff_create: NULL argument");
    if (!same_grid(old_f, new_f))
        return fail(AGAL_EINVAL, "agal_forest_diff_create: forests over different root grids, domains or level counts");
    hipStream_t s = (hipStream_t)stream;
    agal_context ctx = new_f->ctx;
    auto *d = new agal_forest_diff_t;
    d->ctx = ctx;
    d->stream = s;
    d->L = new_f->L;
    unsigned long long *counts = nullptr;
    const int nl = d->L + 1;
    agal_status st = dev_alloc(ctx->mem, &counts, (size_t)nl * 4, s);
    if (st != AGAL_OK) {
        delete d;
        return st;
    }
    fill_u64(reinterpret_cast<uint64_t *>(counts), 0ull, (int64_t)nl * 4, s);
    {
        ProfScope prof(ctx, "forest_diff", s);
        for (int l = 0; l < nl && st == AGAL_OK; ++l) {
            const Level &A = old_f->lev[l], &B = new_f->lev[l];
            d->n_new[l] = B.n;
            d->n_old[l] = A.n;
            st = dev_alloc(ctx->mem, &d->old_index[l], (size_t)std::max<int64_t>(B.n, 1), s);
            if (st == AGAL_OK) st = dev_alloc(ctx->mem, &d->state[l], (size_t)std::max<int64_t>(B.n, 1), s);
            if (st == AGAL_OK) st = dev_alloc(ctx->mem, &d->removed[l], (size_t)std::max<int64_t>(A.n, 1), s);
            if (st != AGAL_OK) break;
            if (B.n > 0)
                hipLaunchKernelGGL(k_diff_new, dim3((unsigned)std::min<int64_t>((B.n + kDiffThreads - 1) / kDiffThreads, 2048)),
                                   dim3(kDiffThreads), 0, s, B.keys, B.leaf, B.n, A.keys, A.leaf, A.n, d->old_index[l],
                                   d->state[l], counts + 4 * l);
            if (A.n > 0)
                hipLaunchKernelGGL(k_diff_old, dim3((unsigned)std::min<int64_t>((A.n + kDiffThreads - 1) / kDiffThreads, 2048)),
                                   dim3(kDiffThreads), 0, s, A.keys, A.n, B.keys, B.n, d->removed[l], counts + 4 * l + 3);
        }
    }
    if (st == AGAL_OK) {
        const hipError_t e1 = hipGetLastError();
        const hipError_t e2 = e1 == hipSuccess ? hipMemcpyAsync(d->counts, counts, (size_t)nl * 4 * 8,
                                                                hipMemcpyDeviceToHost, s)
                                               : e1;
        const hipError_t e3 = e2 == hipSuccess ? hipStreamSynchronize(s) : e2;
        if (e3 != hipSuccess) st = fail(AGAL_EHIP, "agal_forest_diff_create: %s", hipGetErrorString(e3));
    }
    dev_free(ctx->mem, counts, s);
    if (st != AGAL_OK) {
        agal_destroy_forest_diff(d);
        return st;
    }
    *out = d;
    return AGAL_OK;
}

agal_status agal_forest_diff_view(agal_forest_diff d, int level, const int32_t **d_old_index, const uint8_t **d_state,
                                  const uint8_t **d_removed, int64_t *n_new, int64_t *n_old, int64_t counts[4]) {
    if (!d) return fail(AGAL_EINVAL, "agal_forest_diff_view: NULL diff");
    if (level < 0 || level > d->L) return fail(AGAL_EINVAL, "agal_forest_diff_view: level %d outside [0, %d]", level, d->L);
    if (d_old_index) *d_old_index = d->old_index[level];
    if (d_state) *d_state = d->state[level];
    if (d_removed) *d_removed = d->removed[level];
    if (n_new) *n_new = d->n_new[level];
    if (n_old) *n_old = d->n_old[level];
    if (counts)
        for (int k = 0; k < 4; ++k) counts[k] = (int64_t)d->counts[level][k];
    return AGAL_OK;
}

void agal_destroy_forest_diff(agal_forest_diff d) {
    if (!d) return;
    for (int l = 0; l <= kMaxLevels; ++l) {
        dev_free(d->ctx->mem, d->old_index[l], d->stream);
        dev_free(d->ctx->mem, d->state[l], d->stream);
        dev_free(d->ctx->mem, d->removed[l], d->stream);
    }
    delete d;
}

}  // extern "C"
