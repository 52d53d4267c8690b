// Link fractions (paper Sec. II-C-1: cells identify their links with the
// boundary faces along the directions of the velocity set) and their adjoint.
//
// Forward (list mode, the default):
//  * candidate lists: every face lists the finest-level blocks whose link box
//    (block +- one cell) its bounding box meets, found through a hash table of
//    the blocks' parents (a refined block's 2^D children are consecutive in
//    the level); count, exclusive scan, scatter;
//  * node pass: one wave64 per block (four blocks per wave in 2D), one lane
//    per cell, decides which cells have at least one link, stopping at the
//    first certain hit; an exclusive scan of the per-block node counts gives
//    every block its first output row;
//  * row pass: the same waves compute, for the node cells only, the best hit
//    per direction and write each node's row once, at its final place.
//    A wave stages its block's candidate faces in LDS (vertices, FP32 normal,
//    near code), each lane marks the staged faces near its own cell, and
//    (lane, face) pairs go through an FP32 filter with rounding margins over
//    all directions at once; whatever passes is decided, and its t computed,
//    in FP64 with the textbook segment-triangle expressions (FP64 runs at the
//    FP32 rate on this chip, and only near actual hits).
// Walk mode (a face too large for the lists, or lists switched off): one pass
// walks the bins under each block and writes its nodes into the block's own
// slot range of a staging buffer (block * 4^D rows); an exclusive scan of the
// counts and a copy kernel then lay the nodes out in canonical order.
#include <algorithm>
#include <cmath>
#include <vector>

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

// ---- list mode ------------------------------------------------------------
template <int D>
__global__ void k_link_blocks(const uint32_t *keys, int64_t n, unsigned long long *hash, uint32_t hmask, int hshift,
                              unsigned long long *mask) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        link_block_item<D>(keys, i, hash, hmask, hshift, mask);
}

template <int D, bool kScatter>
__global__ __launch_bounds__(64) void k_link_faces(const float *aabb, int64_t F, LinkFaceGrid G, BlockFind B,
                                                   int64_t max_coords, uint32_t *cnt, const uint32_t *loff,
                                                   uint32_t *cursor, int32_t *list, uint32_t *lblk, uint32_t cap) {
    link_faces_wave<D, kScatter>(aabb, F, G, B, max_coords, cnt, loff, cursor, list, lblk, cap,
                                 (int64_t)blockIdx.x * kLinkFaceG);
}

template <int D, int Q>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_links_nodes(LinkArgs<D, Q> A, const uint32_t *lblk,
                                                    unsigned long long *mask) {
    links_nodes_entries<D, Q>(A, lblk, mask, blockIdx.x, gridDim.x);
}

template <int D>
__global__ __launch_bounds__(256) void k_node_map(const unsigned long long *mask, const uint32_t *noff,
                                                  const uint32_t *keys, int64_t n, uint32_t *nblk,
                                                  uint64_t *node_key) {
    // 64 blocks per wave at a time
    const int64_t w0 = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * 256u + threadIdx.x) / 64u));
    for (int64_t c = w0; c * 64 < n; c += (int64_t)gridDim.x * 4)
        node_map_chunk<D>(mask, noff, keys, c * 64, n, nblk, node_key);
}

template <int D, int Q>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_links_rows(
    LinkArgs<D, Q> A, const uint32_t *lblk, const uint32_t *nblk, uint32_t nn) {
    links_rows_nodes<D, Q>(A, lblk, nblk, A.node_key, nn, (int64_t)blockIdx.x);
}

template <int D, int Q>
LinkArgs<D, Q> link_args(agal_geom g, agal_bins bn, agal_forest fo) {
    const agal::Level &LL = fo->lev[fo->L];
    LinkArgs<D, Q> A{};
    A.faces = dev::Faces{g->coords, g->aabb, g->rec, g->F};
    A.bins.off = bn->off;
    A.bins.ids = bn->ids;
    A.bins.B = bn->B;
    A.bins.F = g->F;
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
    return A;
}

// Device memory of one call, released when the call returns (stream ordered).
struct CallScratch {
    agal_context ctx;
    hipStream_t s;
    std::vector<void *> ptrs;
    template <class T>
    agal_status get(T **p, size_t count) {
        AGAL_TRY(dev_alloc(ctx->mem, p, count, s));
        ptrs.push_back(*p);
        return AGAL_OK;
    }
    ~CallScratch() {
        for (void *p : ptrs) dev_free(ctx->mem, p, s);
    }
};

template <int D, int Q>
agal_status alloc_link_outputs(agal_links lk, uint32_t nn, hipStream_t s) {
    agal_context ctx = lk->ctx;
    lk->n = nn;
    AGAL_TRY(dev_alloc(ctx->mem, &lk->key, (size_t)std::max<uint32_t>(nn, 1u), s));
    AGAL_TRY(dev_alloc(ctx->mem, &lk->q, (size_t)std::max<uint32_t>(nn, 1u) * Q, s));
    AGAL_TRY(dev_alloc(ctx->mem, &lk->face, (size_t)std::max<uint32_t>(nn, 1u) * Q, s));
    return AGAL_OK;
}

// Walk mode: bins walked per block, nodes staged per block, then compacted.
template <int D, int Q>
agal_status links_forward_walk(agal_geom g, agal_bins bn, agal_forest fo, agal_links lk, hipStream_t s) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int BPW = 64 / CELLS;
    agal_context ctx = g->ctx;
    const agal::Level &LL = fo->lev[fo->L];
    const int64_t cap = LL.n * CELLS;   // staging rows: every cell of every block
    CallScratch st{ctx, s};
    uint32_t *count = nullptr, *off = nullptr;
    uint64_t *skey = nullptr, *status = nullptr;
    float *sq = nullptr;
    int32_t *sface = nullptr;
    AGAL_TRY(st.get(&count, (size_t)LL.n));
    AGAL_TRY(st.get(&off, (size_t)LL.n + 1));
    AGAL_TRY(st.get(&status, (size_t)scan_tiles(LL.n) + 1));
    AGAL_TRY(st.get(&skey, (size_t)cap));
    AGAL_TRY(st.get(&sq, (size_t)cap * Q));
    AGAL_TRY(st.get(&sface, (size_t)cap * Q));
    LinkArgs<D, Q> A = link_args<D, Q>(g, bn, fo);
    A.node_key = skey;
    A.q = sq;
    A.face = sface;
    const int64_t waves = (LL.n + BPW - 1) / BPW;
    {
        ProfScope prof(ctx, "q_links", s);
        hipLaunchKernelGGL((k_links<D, Q>), dim3((unsigned)waves), dim3(64), 0, s, A, count, status,
                           scan_tiles(LL.n) + 1);
    }
    AGAL_TRY_HIP(hipGetLastError());
    uint32_t nn = 0;
    AGAL_TRY(scan_u32_total(ctx, count, off, LL.n, status, &nn, s));
    AGAL_TRY((alloc_link_outputs<D, Q>(lk, nn, s)));
    if (nn > 0) {
        ProfScope prof(ctx, "q_compact", s);
        hipLaunchKernelGGL((k_compact_nodes<Q, CELLS>), dim3((unsigned)LL.n), dim3(64), 0, s, count, off, LL.n,
                           skey, sq, sface, lk->key, lk->q, lk->face);
    }
    AGAL_TRY_HIP(hipGetLastError());
    return AGAL_OK;
}

// First half of the list build: the parent table, the zeroed node masks and
// every block's candidate count (lwork[0 .. n); lwork[n .. 2n) zeroed for the
// scatter cursors).
template <int D>
struct ListBuild {
    BlockFind B{};
    LinkFaceGrid G{};
    unsigned long long *nmask = nullptr;
    uint32_t *lwork = nullptr;
};

template <int D>
agal_status list_count(agal_geom g, agal_forest fo, const float eps[3], int64_t max_coords, CallScratch &st,
                       ListBuild<D> &LB, hipStream_t s) {
    const agal::Level &LL = fo->lev[fo->L];
    const int64_t n = LL.n;
    const int L = fo->L;
    BlockFind &B = LB.B;
    B.level = L;
    B.keys = LL.keys;
    B.n = n;
    for (int a = 0; a < 3; ++a) B.R[a] = fo->roots[a];
    unsigned long long *hash = nullptr;
    const unsigned fgrid = (unsigned)((g->F + kLinkFaceG - 1) / kLinkFaceG);
    const unsigned bgrid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    AGAL_TRY(st.get(&LB.nmask, (size_t)n));
    if (L > 0) {
        // parents: n / 2^D (complete families); at most half the slots used
        int bits = 6;
        while (bits < 31 && (int64_t(1) << bits) < 2 * ((n + (1 << D) - 1) >> D)) ++bits;
        B.hmask = (uint32_t)((int64_t(1) << bits) - 1);
        B.hshift = 32 - bits;
        AGAL_TRY(st.get(&hash, (size_t)B.hmask + 1));
        fill_u64(reinterpret_cast<uint64_t *>(hash), ~0ull, (int64_t)B.hmask + 1, s);
    }
    hipLaunchKernelGGL((k_link_blocks<D>), dim3(bgrid), dim3(256), 0, s, LL.keys, n, hash, B.hmask, B.hshift,
                       LB.nmask);
    B.hash = hash;
    LinkFaceGrid &G = LB.G;
    for (int a = 0; a < 3; ++a) {
        G.lo[a] = fo->lo[a];
        G.dx[a] = fo->dx[L][a];
        G.m[a] = 2.0 * (double)eps[a];
        G.NB[a] = a < D ? (fo->roots[a] << L) : 1;
    }
    AGAL_TRY(st.get(&LB.lwork, (size_t)2 * n));   // counts, then scatter cursors
    fill_u32(LB.lwork, 0u, 2 * n, s);
    hipLaunchKernelGGL((k_link_faces<D, false>), dim3(fgrid), dim3(64), 0, s, g->aabb, g->F, G, B, max_coords,
                       LB.lwork, nullptr, nullptr, nullptr, nullptr, 0u);
    AGAL_TRY_HIP(hipGetLastError());
    return AGAL_OK;
}

// Link step mode of (g, fo): list mode while every face has few candidate
// blocks and the list fits 32-bit offsets.
struct LinkMode {
    bool lists = false;
    int64_t per_face = 0;   // candidate blocks per face at most
    double cap = 0.0;       // list length bound
    float eps[3] = {0, 0, 0};
};

inline LinkMode link_mode(agal_geom g, agal_forest fo) {
    LinkMode m;
    float dx[3];
    for (int a = 0; a < 3; ++a) {
        dx[a] = fo->dx[fo->L][a];
        m.eps[a] = dev::kEps * std::max(1.0f, std::max(std::fabs(fo->lo[a]), std::fabs(fo->hi[a])));
    }
    const double per_face = link_blocks_per_face(g->dim, g->max_extent, dx, m.eps);
    m.cap = per_face * (double)g->F;
    m.lists = per_face <= (double)g->ctx->link_list_max && m.cap <= (double)UINT32_MAX;
    m.per_face = m.lists ? (int64_t)per_face : 0;
    return m;
}

// List mode: candidate lists, node pass, scan, row pass (rows written once).
// A list bound above kListNoWait entries is replaced by the exact length (one
// more host wait) rather than allocated.
constexpr int64_t kListNoWait = int64_t(1) << 26;

template <int D, int Q>
agal_status links_forward_lists(agal_geom g, agal_bins bn, agal_forest fo, agal_links lk, int64_t max_coords,
                                int64_t list_cap, hipStream_t s) {
    agal_context ctx = g->ctx;
    const agal::Level &LL = fo->lev[fo->L];
    const int64_t n = LL.n;
    LinkArgs<D, Q> A = link_args<D, Q>(g, bn, fo);
    CallScratch st{ctx, s};
    ListBuild<D> LB;
    uint32_t *loff = nullptr, *lblk = nullptr, *noff = nullptr, *nblk = nullptr;
    int32_t *list = nullptr;
    const unsigned fgrid = (unsigned)((g->F + kLinkFaceG - 1) / kLinkFaceG);
    const unsigned bgrid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    {
        ProfScope prof(ctx, "q_lists", s);
        AGAL_TRY(list_count<D>(g, fo, A.eps, max_coords, st, LB, s));
        AGAL_TRY(st.get(&loff, (size_t)n + 1));
        if (list_cap <= kListNoWait) {
            // the bound is small enough to allocate: no host wait
            AGAL_TRY(scan_u32(ctx, LB.lwork, loff, n, s));
        } else {
            uint32_t total = 0;
            AGAL_TRY(scan_u32_total(ctx, LB.lwork, loff, n, nullptr, &total, s));
            list_cap = total;
        }
        AGAL_TRY(st.get(&list, (size_t)std::max<int64_t>(list_cap, 1)));
        AGAL_TRY(st.get(&lblk, (size_t)std::max<int64_t>(list_cap, 1)));
        hipLaunchKernelGGL((k_link_faces<D, true>), dim3(fgrid), dim3(64), 0, s, g->aabb, g->F, LB.G, LB.B,
                           max_coords, nullptr, loff, LB.lwork + n, list, lblk, (uint32_t)list_cap);
    }
    AGAL_TRY_HIP(hipGetLastError());
    A.loff = loff;
    A.list = list;
    A.list_cap = (uint32_t)list_cap;
    unsigned long long *nmask = LB.nmask;
    {
        // persistent waves over the list entries: eight per SIMD at most
        const int64_t want = (list_cap + 63) / 64;
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->n_cu * 4 * 8));
        ProfScope prof(ctx, "q_nodes", s);
        hipLaunchKernelGGL((k_links_nodes<D, Q>), dim3(grid), dim3(64), 0, s, A, lblk, nmask);
    }
    AGAL_TRY_HIP(hipGetLastError());
    AGAL_TRY(st.get(&noff, (size_t)n + 1));
    uint32_t nn = 0;
    AGAL_TRY(scan_popc64_total(ctx, nmask, noff, n, &nn, s));
    AGAL_TRY((alloc_link_outputs<D, Q>(lk, nn, s)));
    if (nn > 0) {
        AGAL_TRY(st.get(&nblk, (size_t)nn));
        A.node_key = lk->key;
        A.q = lk->q;
        A.face = lk->face;
        ProfScope prof(ctx, "q_links", s);
        const unsigned mgrid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
        hipLaunchKernelGGL((k_node_map<D>), dim3(mgrid), dim3(256), 0, s, nmask, noff, LL.keys, n, nblk, lk->key);
        hipLaunchKernelGGL((k_links_rows<D, Q>), dim3((unsigned)(((int64_t)nn + kRowNodes - 1) / kRowNodes)), dim3(64), 0, s, A, lblk,
                           nblk, nn);
    }
    AGAL_TRY_HIP(hipGetLastError());
    return AGAL_OK;
}

template <int D, int Q>
agal_status links_forward(agal_geom g, agal_bins bn, agal_forest fo, const Lattice &, agal_links lk, hipStream_t s) {
    const agal::Level &LL = fo->lev[fo->L];
    if (LL.n == 0) return alloc_link_outputs<D, Q>(lk, 0u, s);
    const LinkMode m = link_mode(g, fo);
    if (m.lists) return links_forward_lists<D, Q>(g, bn, fo, lk, m.per_face, (int64_t)m.cap, s);
    if (bn->discrete)
        return fail(AGAL_EINVAL, "agal_link_fractions: the faces are too large for candidate lists and the bin walk "
                                 "needs bins by bounding box, not by sampled points");
    return links_forward_walk<D, Q>(g, bn, fo, lk, s);
}

template <int D>
agal_status list_entries_impl(agal_geom g, agal_forest fo, const LinkMode &m, int64_t *entries, hipStream_t s) {
    CallScratch st{g->ctx, s};
    ListBuild<D> LB;
    const int64_t n = fo->lev[fo->L].n;
    uint32_t *loff = nullptr;
    AGAL_TRY(list_count<D>(g, fo, m.eps, m.per_face, st, LB, s));
    AGAL_TRY(st.get(&loff, (size_t)n + 1));
    uint32_t total = 0;
    AGAL_TRY(scan_u32_total(g->ctx, LB.lwork, loff, n, nullptr, &total, s, false));
    *entries = total;
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

// ---- node classification ---------------------------------------------------
// Side of each boundary node from the faces its links meet: the faces are
// oriented so that n = (b - a) x (c - a) (3D) or n = (e_y, -e_x) (2D) points
// out of the solid, so a link entering the solid has c_i . n < 0 and one
// leaving it c_i . n > 0.  The sign is taken in FP64 from the face's FP32
// corners (edge differences and the two-term products exact, one rounding per
// normal component and per sum, in a fixed order), so it is the same on every
// device.  First every face gets its signs for all directions at once (bit i:
// c_i . n < 0, bit 32 + i: c_i . n > 0, both for 0), 8 bytes per face; then
// the nodes' rows are read as one flat run of slots, 64 consecutive slots per
// wave and kClassU runs in flight per thread (face ids, then the faces' sign
// words, loaded together).  Every slot whose face has a sign bit for its
// direction ORs its code (1 entering, 2 leaving) into its node's LDS word:
// one LDS atomic instruction per run, its lanes those slots (a node's few
// links meet at one word).
template <int D, int Q>
__global__ __launch_bounds__(256) void k_face_signs(const float *rec, int64_t F, unsigned long long *sign) {
    static_assert(Q <= 32, "direction bits in 32-bit halves");
    for (int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x; f < F; f += (int64_t)gridDim.x * 256) {
        float w[dev::kRecFloats<D>];
        dev::load_rec<D>(rec, f, w);
        double nrm[3] = {0.0, 0.0, 0.0};
        if constexpr (D == 3) {
            const double e1[3] = {(double)w[3] - (double)w[0], (double)w[4] - (double)w[1], (double)w[5] - (double)w[2]};
            const double e2[3] = {(double)w[6] - (double)w[0], (double)w[7] - (double)w[1], (double)w[8] - (double)w[2]};
            nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
            nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
            nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
        } else {
            nrm[0] = (double)w[3] - (double)w[1];
            nrm[1] = -((double)w[2] - (double)w[0]);
        }
        uint32_t enter = 0u, leave = 0u;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const double sg = ((double)dir_c<D>(i, 0) * nrm[0] + (double)dir_c<D>(i, 1) * nrm[1]) +
                              (double)dir_c<D>(i, 2) * nrm[2];
            enter |= sg <= 0.0 ? (1u << i) : 0u;
            leave |= sg >= 0.0 ? (1u << i) : 0u;
        }
        sign[f] = ((unsigned long long)leave << 32) | enter;
    }
}

constexpr int kClassThreads = 256;
constexpr int kClassU = 4;

template <int Q>
__global__ __launch_bounds__(kClassThreads) void k_classify_nodes(const unsigned long long *sign, int64_t F,
                                                                  const int32_t *face, int64_t n, uint8_t *cls) {
    __shared__ uint32_t s_code[kClassThreads];
    const int tid = threadIdx.x;
    const int lane = dev::lane_id();
    const int64_t node0 = (int64_t)blockIdx.x * kClassThreads;
    const int nn = (int)min((int64_t)kClassThreads, n - node0);
    s_code[tid] = 0u;
    __syncthreads();
    const int span = nn * Q;
    const int32_t *row = face + node0 * Q;
    // slot sl = k0 + u kClassThreads + tid: node sl / Q, direction sl % Q,
    // advanced by kClassThreads slots a step
    constexpr int SN = kClassThreads / Q, SI = kClassThreads % Q;
    int node = tid / Q, i = tid - (tid / Q) * Q;
    for (int k0 = 0; k0 < span; k0 += kClassU * kClassThreads) {
        int32_t f[kClassU];
#pragma unroll
        for (int u = 0; u < kClassU; ++u) {
            const int sl = k0 + u * kClassThreads + tid;
            f[u] = sl < span ? row[sl] : -1;
        }
        unsigned long long t[kClassU];
#pragma unroll
        for (int u = 0; u < kClassU; ++u) t[u] = f[u] >= 0 && f[u] < F ? sign[f[u]] : 0ull;
#pragma unroll
        for (int u = 0; u < kClassU; ++u) {
            // the slot's code: 1 when its link enters the body through the face, 2 when it leaves
            // (the rest direction, i = 0, has bit 0 clear in both halves; slots past the span have t = 0)
            const uint32_t c = (uint32_t)((t[u] >> i) & 1ull) | ((uint32_t)((t[u] >> (32 + i)) & 1ull) << 1);
            if (c) atomicOr(&s_code[node], c);
            node += SN;
            i += SI;
            if (i >= Q) {
                i -= Q;
                ++node;
            }
        }
    }
    __syncthreads();
    if (tid < nn) {
        const uint32_t c = s_code[tid];
        cls[node0 + tid] = (uint8_t)(c == 3u ? 3u : (c == 2u ? 2u : 1u));
    }
}

template <int D, int Q>
agal_status classify_nodes(agal_geom g, agal_links lk, uint8_t *cls, hipStream_t s) {
    if (lk->n == 0) return AGAL_OK;
    CallScratch st{g->ctx, s};
    unsigned long long *sign = nullptr;
    AGAL_TRY(st.get(&sign, (size_t)std::max<int64_t>(g->F, 1)));
    const int64_t blocks = (lk->n + kClassThreads - 1) / kClassThreads;
    {
        ProfScope prof(g->ctx, "classify", s);
        hipLaunchKernelGGL((k_face_signs<D, Q>), dim3((unsigned)std::min<int64_t>((g->F + 255) / 256, 8192)),
                           dim3(256), 0, s, g->rec, g->F, sign);
        hipLaunchKernelGGL((k_classify_nodes<Q>), dim3((unsigned)blocks), dim3(kClassThreads), 0, s, sign, g->F,
                           lk->face, lk->n, cls);
    }
    AGAL_TRY_HIP(hipGetLastError());
    return AGAL_OK;
}

}  // namespace

agal_status link_list_plan(agal_geom g, agal_forest fo, hipStream_t s, LinkListPlan *out) {
    *out = LinkListPlan{};
    const LinkMode m = link_mode(g, fo);
    out->lists = m.lists && fo->lev[fo->L].n > 0;
    if (!out->lists) return AGAL_OK;
    out->per_face = m.per_face;
    if (g->dim == 3) return list_entries_impl<3>(g, fo, m, &out->entries, s);
    return list_entries_impl<2>(g, fo, m, &out->entries, s);
}

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

agal_status agal_classify_nodes(agal_geom g, agal_links l, uint8_t *d_class, void *stream) {
    if (!g || !l) return fail(AGAL_EINVAL, "agal_classify_nodes: NULL handle");
    if (l->geom_id != g->id) return fail(AGAL_ESTATE, "agal_classify_nodes: links were computed from another geometry");
    if (l->n > 0 && !d_class) return fail(AGAL_EINVAL, "agal_classify_nodes: NULL output");
    if (l->n > (int64_t)kClassThreads * INT32_MAX) return fail(AGAL_EINVAL, "agal_classify_nodes: too many nodes");
    hipStream_t s = (hipStream_t)stream;
    if (l->Q == AGAL_D2Q9) return classify_nodes<2, 9>(g, l, d_class, s);
    if (l->Q == AGAL_D3Q19) return classify_nodes<3, 19>(g, l, d_class, s);
    return classify_nodes<3, 27>(g, l, d_class, s);
}

void agal_destroy_links(agal_links l) {
    if (!l) return;
    dev_free(l->ctx->mem, l->key, l->stream);
    dev_free(l->ctx->mem, l->q, l->stream);
    dev_free(l->ctx->mem, l->face, l->stream);
    delete l;
}

}  // extern "C"
