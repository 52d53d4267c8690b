// Link fractions (paper Sec. II-C-1: cells identify their links with the
// boundary faces along the directions of the velocity set) and their adjoint.
//
// Forward, one wave64 per finest-level block (four blocks per wave in 2D),
// one lane per cell:
//  * the wave gathers the faces of the bins under the block's link box
//    (block +- one cell), culls them by bounding box and stages, per face,
//    vertices a, b, c, the FP32 normal n = (b - a) x (c - a) and the bounding
//    box in LDS;
//  * each lane culls every staged face against its own link box, then
//    filters all directions at once in FP32.  With T = o - a, E1 = b - a,
//    E2 = c - a the solution of o + t D = a + u E1 + v E2 is
//        det = D.n,  u = D.(T x E2)/det,  v = D.(E1 x T)/det,  t = -(T.n)/det;
//    T x E2, E1 x T and T.n do not depend on D, and D = c_i dx has entries
//    in {-dx, 0, dx}, so a direction costs a few additions, and the opposite
//    direction has the same u, v and t of the opposite sign, so directions
//    are handled in +/- pairs.  The filter widens every test by a bound on
//    its FP32 rounding error; whatever passes is decided, and its t computed,
//    in FP64 with the textbook segment-triangle expressions (FP64 runs at the
//    FP32 rate on this chip, and only near actual hits);
//  * cells with at least one link are written to their block's own slot range
//    of a staging buffer (block * 4^D rows), with the block's node count; an
//    exclusive scan of the counts and a copy kernel then lay the nodes out in
//    canonical order.  (An in-kernel ordered prefix would make every wave wait
//    for its slowest predecessor before it could publish its count.)
#include <algorithm>
#include <cmath>

#include "agal_internal.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace agal {
namespace {

using namespace kern;

// Staging rows of block b start at b * 4^D; its node count goes to count[b].
template <int CELLS>
struct BlockSlots {
    uint32_t *count;
    __device__ int64_t rows(int64_t blk, uint32_t c) {
        count[blk] = c;
        return blk * CELLS;
    }
};

template <int D, int Q>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_links(LinkArgs<D, Q> A, uint32_t *count, uint64_t *zero,
                                                                                           int64_t nzero) {
    // the look-back status words of the scan that follows, cleared here
    // rather than by a launch of their own
    for (int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x; i < nzero; i += (int64_t)gridDim.x * 64) zero[i] = 0;
    BlockSlots<D == 3 ? 64 : 16> out{count};
    links_wave<D, Q>(A, (int64_t)blockIdx.x * (D == 3 ? 1 : 4), out);
}

template <int D, int Q>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint(AdjArgs<D, Q> A) {
    adjoint_tile<D, Q>(A, (int64_t)blockIdx.x * kAdjThreads);
}

// Staged nodes of block b (rows b*4^D .. b*4^D + count[b]) -> rows off[b].. of
// the output; one wave per block, rows copied as flat coalesced runs.
template <int Q, int CELLS>
__global__ __launch_bounds__(64) void k_compact_nodes(const uint32_t *count, const uint32_t *off, int64_t nblk,
                                                      const uint64_t *skey, const float *sq, const int32_t *sface,
                                                      uint64_t *key, float *q, int32_t *face) {
    const int64_t b = blockIdx.x;
    if (b >= nblk) return;
    compact_block<Q>((int)count[b], b * CELLS, off[b], skey, sq, sface, key, q, face);
}

template <int D, int Q>
agal_status links_forward(agal_geom g, agal_bins bn, agal_forest fo, const Lattice &lat, agal_links lk, hipStream_t s) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int BPW = 64 / CELLS;
    agal_context ctx = g->ctx;
    const agal::Level &LL = fo->lev[fo->L];
    if (LL.n == 0) {
        AGAL_TRY(dev_alloc(ctx->mem, &lk->key, 1, s));
        AGAL_TRY(dev_alloc(ctx->mem, &lk->q, (size_t)Q, s));
        AGAL_TRY(dev_alloc(ctx->mem, &lk->face, (size_t)Q, s));
        lk->n = 0;
        return AGAL_OK;
    }
    const int64_t cap = LL.n * CELLS;   // staging rows: every cell of every block
    struct Staging {
        agal_context ctx;
        hipStream_t s;
        uint32_t *count = nullptr, *off = nullptr;
        uint64_t *key = nullptr, *status = nullptr;
        float *q = nullptr;
        int32_t *face = nullptr;
        ~Staging() {
            dev_free(ctx->mem, status, s);
            dev_free(ctx->mem, count, s);
            dev_free(ctx->mem, off, s);
            dev_free(ctx->mem, key, s);
            dev_free(ctx->mem, q, s);
            dev_free(ctx->mem, face, s);
        }
    } st{ctx, s};
    AGAL_TRY(dev_alloc(ctx->mem, &st.count, (size_t)LL.n, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.off, (size_t)LL.n + 1, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.status, (size_t)scan_tiles(LL.n) + 1, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.key, (size_t)cap, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.q, (size_t)cap * Q, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.face, (size_t)cap * Q, s));
    LinkArgs<D, Q> A{};
    A.faces = dev::Faces{g->coords, g->aabb, g->rec, g->F};
    A.bins.off = bn->off;
    A.bins.ids = bn->ids;
    A.bins.B = bn->B;
    for (int a = 0; a < 3; ++a) {
        A.bins.lo[a] = bn->lo[a];
        A.bins.s[a] = bn->s[a];
        A.R[a] = fo->roots[a];
        A.lo[a] = fo->lo[a];
        A.dx[a] = fo->dx[fo->L][a];
        float sc = std::max(1.0f, std::max(std::fabs(fo->lo[a]), std::fabs(fo->hi[a])));
        A.eps[a] = dev::kEps * sc;
    }
    A.keys = LL.keys;
    A.n = LL.n;
    A.level = fo->L;
    A.node_key = st.key;
    A.q = st.q;
    A.face = st.face;
    const int64_t waves = (LL.n + BPW - 1) / BPW;
    {
        ProfScope prof(ctx, "q_links", s);
        hipLaunchKernelGGL((k_links<D, Q>), dim3((unsigned)waves), dim3(64), 0, s, A, st.count, st.status,
                           scan_tiles(LL.n) + 1);
    }
    AGAL_TRY_HIP(hipGetLastError());
    uint32_t nn = 0;
    AGAL_TRY(scan_u32_total(ctx, st.count, st.off, LL.n, st.status, &nn, s));
    lk->n = nn;
    AGAL_TRY(dev_alloc(ctx->mem, &lk->key, (size_t)std::max<uint32_t>(nn, 1u), s));
    AGAL_TRY(dev_alloc(ctx->mem, &lk->q, (size_t)std::max<uint32_t>(nn, 1u) * Q, s));
    AGAL_TRY(dev_alloc(ctx->mem, &lk->face, (size_t)std::max<uint32_t>(nn, 1u) * Q, s));
    if (nn > 0) {
        ProfScope prof(ctx, "q_compact", s);
        hipLaunchKernelGGL((k_compact_nodes<Q, CELLS>), dim3((unsigned)LL.n), dim3(64), 0, s, st.count, st.off, LL.n,
                           st.key, st.q, st.face, lk->key, lk->q, lk->face);
    }
    AGAL_TRY_HIP(hipGetLastError());
    return AGAL_OK;
}

template <int D, int Q>
agal_status links_backward(agal_geom g, agal_links lk, const Lattice &lat, const float *gq, float *grad, hipStream_t s) {
    if (lk->n == 0) return AGAL_OK;
    AdjArgs<D, Q> A{};
    A.rec = g->rec;
    A.F = g->F;
    A.fidx = g->fidx;
    A.node_key = lk->key;
    A.face = lk->face;
    A.gq = gq;
    A.n = lk->n;
    A.level = lk->L;
    for (int a = 0; a < 3; ++a) {
        A.R[a] = lk->roots[a];
        A.lo[a] = lk->lo[a];
        A.dx[a] = lk->dx[a];
    }
    A.grad = grad;
    const int64_t blocks = (lk->n + kAdjThreads - 1) / kAdjThreads;
    {
        ProfScope prof(g->ctx, "q_adjoint", s);
        hipLaunchKernelGGL((k_adjoint<D, Q>), dim3((unsigned)blocks), dim3(kAdjThreads), 0, s, A);
    }
    AGAL_TRY_HIP(hipGetLastError());
    return AGAL_OK;
}

}  // namespace
}  // namespace agal

using namespace agal;

extern "C" {

agal_status agal_link_fractions(agal_geom g, agal_bins b, agal_forest f, int lattice, void *stream, agal_links *out) {
    if (!g || !b || !f || !out) return fail(AGAL_EINVAL, "agal_link_fractions: NULL argument");
    if (b->geom_id != g->id || f->geom_id != g->id)
        return fail(AGAL_ESTATE, "agal_link_fractions: bins or forest built from another geometry");
    Lattice lat;
    if (!lattice_table(lattice, &lat)) return fail(AGAL_EINVAL, "agal_link_fractions: unknown lattice %d", lattice);
    if (lat.dim != g->dim)
        return fail(AGAL_EINVAL, "agal_link_fractions: lattice D%dQ%d does not match dim %d", lat.dim, lattice, g->dim);
    hipStream_t s = (hipStream_t)stream;
    auto *lk = new (std::nothrow) agal_links_t();
    if (!lk) return fail(AGAL_ENOMEM, "agal_link_fractions: host allocation failed");
    lk->ctx = g->ctx;
    lk->geom_id = g->id;
    lk->stream = s;
    lk->dim = g->dim;
    lk->Q = lattice;
    lk->L = f->L;
    for (int a = 0; a < 3; ++a) {
        lk->roots[a] = f->roots[a];
        lk->lo[a] = f->lo[a];
        lk->dx[a] = f->dx[f->L][a];
    }
    agal_status st;
    if (lattice == AGAL_D2Q9) st = links_forward<2, 9>(g, b, f, lat, lk, s);
    else if (lattice == AGAL_D3Q19) st = links_forward<3, 19>(g, b, f, lat, lk, s);
    else st = links_forward<3, 27>(g, b, f, lat, lk, s);
    if (st != AGAL_OK) {
        agal_destroy_links(lk);
        return st;
    }
    *out = lk;
    return AGAL_OK;
}

agal_status agal_links_view(agal_links l, const uint64_t **d_node_key, const float **d_q, const int32_t **d_face,
                            int64_t *n_nodes, int *Q) {
    if (!l) return fail(AGAL_EINVAL, "agal_links_view: NULL links");
    if (d_node_key) *d_node_key = l->key;
    if (d_q) *d_q = l->q;
    if (d_face) *d_face = l->face;
    if (n_nodes) *n_nodes = l->n;
    if (Q) *Q = l->Q;
    return AGAL_OK;
}

agal_status agal_link_fractions_backward(agal_geom g, agal_links l, const float *d_grad_q, float *d_grad_vertices,
                                         void *stream) {
    if (!g || !l) return fail(AGAL_EINVAL, "agal_link_fractions_backward: NULL handle");
    if (l->geom_id != g->id) return fail(AGAL_ESTATE, "agal_link_fractions_backward: links were computed from another geometry");
    if (l->n > 0 && (!d_grad_q || !d_grad_vertices))
        return fail(AGAL_EINVAL, "agal_link_fractions_backward: NULL gradient buffer");
    Lattice lat;
    lattice_table(l->Q, &lat);
    hipStream_t s = (hipStream_t)stream;
    if (l->Q == AGAL_D2Q9) return links_backward<2, 9>(g, l, lat, d_grad_q, d_grad_vertices, s);
    if (l->Q == AGAL_D3Q19) return links_backward<3, 19>(g, l, lat, d_grad_q, d_grad_vertices, s);
    return links_backward<3, 27>(g, l, lat, d_grad_q, d_grad_vertices, s);
}

void agal_destroy_links(agal_links l) {
    if (!l) return;
    dev_free(l->ctx->mem, l->key, l->stream);
    dev_free(l->ctx->mem, l->q, l->stream);
    dev_free(l->ctx->mem, l->face, l->stream);
    delete l;
}

}  // extern "C"
