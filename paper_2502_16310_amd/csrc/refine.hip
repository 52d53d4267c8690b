// Near-wall refinement (paper Sec. II-C-1, II-C-2; forest layout Sec. II-A).
//
// Level by level: every cell of every block of the tested level checks the
// faces of the bins its query box overlaps (the paper's "primary mode of
// access": one level at a time, the block's cells processed together); a
// block with a flagged cell is marked, 2:1 balance marks the coarser
// neighbours that must follow, and marked blocks are replaced by 2^D children
// merged into the next level's sorted key list.
//
// Mapping on CDNA: one wave64 per 4x4x4 block (one lane per cell; four 4x4
// blocks per wave in 2D).  The wave walks the bins under the block's query
// box, culls each face against the box by its bounding box (lane-parallel,
// one face per lane), compacts the survivors with a ballot into LDS, then
// every lane runs the separating-axis test of its cell against the staged
// faces (LDS broadcast reads) and stops once flagged.
#include <algorithm>
#include <cmath>
#include <vector>

#include "agal_internal.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace agal {
namespace {

using namespace kern;

#define AGAL_GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

template <int D, bool kDedup>
__global__ __launch_bounds__(64) void k_flag(FlagArgs<D> A) {
    flag_wave<D, kDedup>(A, (int64_t)blockIdx.x * (D == 3 ? 1 : 4));
}

template <int D>
__global__ __launch_bounds__(64) void k_flag_own_bin(FlagArgs<D> A) {
    flag_own_bin_wave<D>(A, (int64_t)blockIdx.x * (D == 3 ? 1 : 4));
}

template <int D>
__global__ void k_prop_spread(const uint32_t *keys, int64_t n, uint8_t *pm, int l, int R0, int R1, int R2) {
    AGAL_GRID_STRIDE(t, n * (D == 3 ? 26 : 8)) prop_spread_item<D>(keys, n, pm, l, R0, R1, R2, t);
}

__global__ void k_prop_commit(uint8_t *pm, int64_t n) {
    AGAL_GRID_STRIDE(i, n) if (pm[i] == 4) pm[i] = 3;
}

template <int D, int G>
__global__ __launch_bounds__(64 * kFaceFlagWaves) void k_flag_faces(FaceFlagArgs<D> A) {
    __shared__ float s_rec[kFaceFlagWaves][G][dev::kRecFloats<D>];
    __shared__ int s_i[kFaceFlagWaves][G][kFaceFlagInts];
    const int w = (int)threadIdx.x / dev::kWave;
    flag_faces_wave<D, G>(A, ((int64_t)blockIdx.x * kFaceFlagWaves + w) * G, s_rec[w], s_i[w]);
}

template <int D, int G>
void launch_flag_faces(const FaceFlagArgs<D> &A, hipStream_t s) {
    const int64_t per_wg = (int64_t)kFaceFlagWaves * G;
    hipLaunchKernelGGL((k_flag_faces<D, G>), dim3((unsigned)((A.F + per_wg - 1) / per_wg)), dim3(64 * kFaceFlagWaves),
                       0, s, A);
}

// table[block grid position] = block index for every block of a level, the
// block's cell flags zeroed (4^D bytes, 16-byte stores), and the pass's zeroed
// scratch (zero[0 .. nzero)) cleared, in one launch.
template <int D>
__global__ void k_block_table(const uint32_t *keys, int64_t n, int level, int R0, int R1, int NB0, int NB1,
                              uint32_t *table, uint4 *cf, uint32_t *zero, int64_t nzero) {
    constexpr int V = (D == 3 ? 64 : 16) / 16;
    AGAL_GRID_STRIDE(i, n) {
        int c[3];
        dev::decode_key<D>(keys[i], level, R0, R1, c);
        table[((int64_t)c[2] * NB1 + c[1]) * NB0 + c[0]] = (uint32_t)i;
#pragma unroll
        for (int j = 0; j < V; ++j) cf[i * V + j] = make_uint4(0u, 0u, 0u, 0u);
    }
    AGAL_GRID_STRIDE(i, nzero) zero[i] = 0u;
}

template <int D>
__global__ void k_ripple(const uint32_t *keys_m, int64_t n_m, const uint8_t *pm_m, int m, const uint32_t *keys_p,
                         int64_t n_p, const uint8_t *leaf_p, uint8_t *pm_p, int R0, int R1, int R2, uint32_t *err) {
    AGAL_GRID_STRIDE(t, n_m * (D == 3 ? 26 : 8))
    ripple_item<D>(keys_m, n_m, pm_m, m, keys_p, n_p, leaf_p, pm_p, R0, R1, R2, err, t);
}

// Level 0 (every root, key = x-fastest linear index, all leaves, no marks) and
// the error word, in one launch.
// (cf: the roots' cell flags to zero, cf_vec 16-byte words per root, or null;
// zero[0 .. nzero): the first pass's zeroed scratch)
__global__ void k_init_roots(uint32_t *keys, uint8_t *leaf, uint8_t *mark, int64_t n, uint32_t *err, uint4 *cf,
                             int cf_vec, uint32_t *zero, int64_t nzero) {
    AGAL_GRID_STRIDE(i, n) {
        keys[i] = (uint32_t)i;
        leaf[i] = 1;
        mark[i] = 0;
        if (cf)
            for (int j = 0; j < cf_vec; ++j) cf[i * cf_vec + j] = make_uint4(0u, 0u, 0u, 0u);
    }
    AGAL_GRID_STRIDE(i, nzero) zero[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0u;
}

// Child generation of one pass for every parent level m with marks, in two
// launches: first the parents (k_mark_parents_all), then the new child levels
// (existing children moved and new children written, k_grow_all).  Segment i
// is parent level seg[i].m; items of the launches are numbered across the
// segments by the host-made prefixes.
struct GrowSeg {
    const uint32_t *pkeys;   // parent level m
    const uint8_t *pm;
    const uint32_t *pos;
    uint8_t *pleaf, *pmark;
    int64_t pn;
    uint32_t *mk;            // marked parent keys (c of them)
    int64_t c;
    const uint32_t *ckeys;   // child level m + 1 before the pass
    const uint8_t *cleaf, *cmark, *ccf;
    int64_t cn;
    uint32_t *nkeys;         // child level m + 1 after the pass
    uint8_t *nleaf, *nmark, *ncf;
};
struct GrowArgs {
    GrowSeg seg[kMaxLevels + 1];
    int64_t pre_p[kMaxLevels + 2];   // prefix of pn
    int64_t pre_g[kMaxLevels + 2];   // prefix of cn + (c << D)
    int nseg;
    int D;
};

__device__ __forceinline__ int seg_of(const int64_t *pre, int nseg, int64_t i) {
    int k = 0;
    while (k + 1 < nseg && pre[k + 1] <= i) ++k;
    return k;
}

__global__ void k_mark_parents_all(GrowArgs a) {
    AGAL_GRID_STRIDE(i, a.pre_p[a.nseg]) {
        const int k = seg_of(a.pre_p, a.nseg, i);
        const GrowSeg &g = a.seg[k];
        mark_parents_item(g.pkeys, g.pm, g.pos, g.pleaf, g.pmark, g.mk, i - a.pre_p[k]);
    }
}

template <int CELLS>
__global__ void k_grow_all(GrowArgs a) {
    AGAL_GRID_STRIDE(i, a.pre_g[a.nseg]) {
        const int k = seg_of(a.pre_g, a.nseg, i);
        const GrowSeg &g = a.seg[k];
        const int64_t j = i - a.pre_g[k];
        if (j < g.cn)
            merge_old_item<CELLS>(g.ckeys, g.cleaf, g.cmark, g.ccf, g.mk, g.c, a.D, g.nkeys, g.nleaf, g.nmark, g.ncf, j);
        else
            children_item<CELLS>(g.mk, g.ckeys, g.cn, a.D, g.nkeys, g.nleaf, g.nmark, g.ncf, j - g.cn);
    }
}

unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 16384) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

struct Scratch {
    agal_context ctx;
    hipStream_t s;
    std::vector<void *> ptrs;
    template <class T>
    agal_status get(T **p, size_t n) {
        AGAL_TRY(dev_alloc(ctx->mem, p, n, s));
        ptrs.push_back(*p);
        return AGAL_OK;
    }
    ~Scratch() {
        for (void *p : ptrs) ctx->mem.release(p, s);
    }
};

// Which candidate walker the flag pass of n blocks takes at cell size dx and
// distance h.  The deduplicating one (many list entries per memory latency,
// repeats dropped by a hash set before any record is read) shortens the waves
// of blocks whose query box (4 dx + 2 h per axis) spans many bins; it pays for
// clearing the set and for more LDS per wave.  Measured on MI355X: it wins
// when the pass is bound by its longest waves (few blocks: the two coarsest
// levels over a 20,480-face sphere, 4096 and 3776 blocks, 80 -> 60 and
// 40 -> 27 us) and loses when the pass has blocks enough to fill the GPU many
// times (32768 blocks over a 327,680-face body: 285 -> 375 us).
template <int D>
bool flag_dedup(const agal_bins_t *bn, const float dx[3], float h, int64_t n_blocks, int n_cu) {
    double nbins = 1.0;
    for (int a = 0; a < D; ++a) nbins *= std::min((double)bn->B, std::floor((4.0 * dx[a] + 2.0 * h) * bn->s[a]) + 2.0);
    return nbins > 64.0 && n_blocks < 32 * (int64_t)n_cu;
}

// The flag pass of level l runs face-centric (one lane per (face, cell) pair
// near the face) while the level's block grid has at most the context's
// flag_table_max positions (the table is needed above level 0 only) and the
// largest face has at most kFaceFlagMaxPairs candidate cells, else
// cell-centric (one wave per block).  Measured on MI355X, face-centric wins at
// every level tried: flags 127 -> 74 us over a 20,480-face sphere (3 levels)
// and 875 -> 272 us over a 327,680-face body (4 levels), most at the coarse
// levels, whose few blocks each span hundreds of bins.
template <int D>
int64_t block_grid_size(const agal_forest_t *fo, int l) {
    int64_t e = 1;
    for (int a = 0; a < D; ++a) e *= (int64_t)fo->roots[a] << l;
    return e;
}

// Propagation steps of an own-bin pass (Sec. II-C-3): one more than the whole
// number of block lengths in the distance, 1 + floor(d / (4 dx)) with the
// smallest cell size over the axes (FP32); none with one bin, where every cell
// sees every face.  n_prop >= 0 overrides the rule.
inline int prop_steps(const agal_forest_t *fo, int l, int B, int n_prop) {
    if (n_prop >= 0) return n_prop;
    if (B <= 1) return 0;
    float dxm = fo->dx[l][0];
    for (int a = 1; a < fo->dim; ++a) dxm = std::min(dxm, fo->dx[l][a]);
    return 1 + (int)std::floor(fo->d[l] / (4.0f * dxm));
}

template <int D>
agal_status refine_impl(agal_geom g, agal_bins bn, agal_forest fo, hipStream_t s, bool own_bin = false,
                        int n_prop = -1) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int BPW = 64 / CELLS;
    agal_context ctx = g->ctx;
    const auto &mem = ctx->mem;
    uint32_t *err = nullptr;
    Scratch keep{ctx, s, {}};
    AGAL_TRY(keep.get(&err, 1));

    // level 0: every root, key = x-fastest linear index
    agal::Level &L0 = fo->lev[0];
    L0.n = (int64_t)fo->roots[0] * fo->roots[1] * fo->roots[2];
    AGAL_TRY(dev_alloc(mem, &L0.keys, (size_t)L0.n, s));
    AGAL_TRY(dev_alloc(mem, &L0.leaf, (size_t)L0.n, s));
    AGAL_TRY(dev_alloc(mem, &L0.mark, (size_t)L0.n, s));
    // Zeroed scratch of pass l: the look-back status words of the pass's scan of
    // the marks, then the pass marks of every level l' <= l.
    struct PassBuf {
        uint8_t *buf = nullptr;
        int64_t words = 0, status_bytes = 0;
    };
    auto pass_buf = [&](Scratch &sc, int l, PassBuf &pb) -> agal_status {
        int64_t ns[kMaxLevels + 1], tot = 0;
        for (int m = 0; m <= l; ++m) {
            ns[m] = fo->lev[m].n;
            tot += ns[m];
        }
        pb.status_bytes = 8 * (scan_flags_u8_multi_tiles(ns, l + 1) + 1);
        pb.words = (pb.status_bytes + tot + 3) / 4;
        return sc.get(&pb.buf, (size_t)(4 * pb.words));
    };
    // the level-0 cell flags (for the face-centric step) and the first pass's
    // scratch are zeroed by the root-init launch
    PassBuf pb0;
    if (fo->L > 0) {
        AGAL_TRY(dev_alloc(mem, &L0.cf, (size_t)L0.n * CELLS, s));
        AGAL_TRY(pass_buf(keep, 0, pb0));
    }
    hipLaunchKernelGGL(k_init_roots, dim3(grid_for(L0.n)), dim3(256), 0, s, L0.keys, L0.leaf, L0.mark, L0.n, err,
                       reinterpret_cast<uint4 *>(L0.cf), CELLS / 16, reinterpret_cast<uint32_t *>(pb0.buf),
                       pb0.words);

    dev::BinGrid bins{};
    bins.off = bn->off;
    bins.ids = bn->ids;
    bins.B = bn->B;
    bins.F = g->F;
    for (int a = 0; a < 3; ++a) {
        bins.lo[a] = bn->lo[a];
        bins.s[a] = bn->s[a];
    }
    dev::Faces faces{g->coords, g->aabb, g->rec, g->F};

    for (int l = 0; l < fo->L; ++l) {
        Scratch pass{ctx, s, {}};
        agal::Level &Ll = fo->lev[l];
        float eps_l[3];
        for (int a = 0; a < 3; ++a) eps_l[a] = dev::kEps * std::max(1.0f, std::max(std::fabs(fo->lo[a]), std::fabs(fo->hi[a])));
        const bool by_face = !own_bin && block_grid_size<D>(fo, l) <= ctx->flag_table_max &&
                             face_flag_pairs(D, g->max_extent, fo->d[l], fo->dx[l], eps_l) <= kFaceFlagMaxPairs;
        // the block table of level l (face-centric step above level 0): never
        // cleared, its entries are checked against the level's keys
        uint32_t *table = nullptr;
        if (l > 0 && by_face && Ll.n > 0) AGAL_TRY(pass.get(&table, (size_t)block_grid_size<D>(fo, l)));
        PassBuf pb = pb0;
        if (l > 0) {
            AGAL_TRY(pass_buf(pass, l, pb));
            // zeroed by the table launch when there is one
            if (!table) fill_u32(reinterpret_cast<uint32_t *>(pb.buf), 0u, pb.words, s);
        }
        uint8_t *pm[kMaxLevels + 1] = {};
        uint64_t *scan_status = reinterpret_cast<uint64_t *>(pb.buf);
        {
            int64_t at = pb.status_bytes;
            for (int m = 0; m <= l; ++m) {
                pm[m] = pb.buf + at;
                at += fo->lev[m].n;
            }
        }
        // (i) flag every cell of every level-l block
        if (l > 0) AGAL_TRY(dev_alloc(mem, &Ll.cf, (size_t)Ll.n * CELLS, s));
        if (Ll.n > 0) {
            FlagArgs<D> A{};
            A.faces = faces;
            A.bins = bins;
            A.keys = Ll.keys;
            A.n = Ll.n;
            A.level = l;
            for (int a = 0; a < 3; ++a) {
                A.R[a] = fo->roots[a];
                A.lo[a] = fo->lo[a];
                A.dx[a] = fo->dx[l][a];
                float sc = std::max(1.0f, std::max(std::fabs(fo->lo[a]), std::fabs(fo->hi[a])));
                A.eps[a] = dev::kEps * sc;
            }
            A.h = fo->d[l];
            A.cf = Ll.cf;
            A.pmark = pm[l];
            const int64_t waves = (Ll.n + BPW - 1) / BPW;
            ProfScope prof(ctx, "flag_sat", s);
            const bool dedup = flag_dedup<D>(bn, fo->dx[l], A.h, Ll.n, ctx->n_cu);
            if (own_bin) {
                hipLaunchKernelGGL((k_flag_own_bin<D>), dim3((unsigned)waves), dim3(64), 0, s, A);
            } else if (by_face) {
                FaceFlagArgs<D> B{};
                B.rec = g->rec;
                B.F = g->F;
                for (int a = 0; a < 3; ++a) {
                    B.NB[a] = a < D ? fo->roots[a] << l : 1;
                    B.lo[a] = A.lo[a];
                    B.dx[a] = A.dx[a];
                    B.eps[a] = A.eps[a];
                }
                B.table = table;
                B.keys = Ll.keys;
                B.n = Ll.n;
                B.level = l;
                B.R[0] = fo->roots[0];
                B.R[1] = fo->roots[1];
                B.h = A.h;
                B.cf = Ll.cf;
                B.pmark = pm[l];
                // the cell flags start at zero: level 0's from k_init_roots, the others' here
                if (table)
                    hipLaunchKernelGGL(k_block_table<D>, dim3(grid_for(Ll.n)), dim3(256), 0, s, Ll.keys, Ll.n, l,
                                       fo->roots[0], fo->roots[1], B.NB[0], B.NB[1], table,
                                       reinterpret_cast<uint4 *>(Ll.cf), reinterpret_cast<uint32_t *>(pb.buf),
                                       pb.words);
                if (g->F > 0) {
                    const int G = face_flag_g(g->F, ctx->n_cu);
                    if (G == 16) launch_flag_faces<D, 16>(B, s);
                    else if (G == 8) launch_flag_faces<D, 8>(B, s);
                    else launch_flag_faces<D, 4>(B, s);
                }
            } else if (dedup) {
                hipLaunchKernelGGL((k_flag<D, true>), dim3((unsigned)waves), dim3(64), 0, s, A);
            } else {
                hipLaunchKernelGGL((k_flag<D, false>), dim3((unsigned)waves), dim3(64), 0, s, A);
            }
        }
        // (i') own-bin pass: the marks spread over prop_steps rings of level-l blocks
        if (own_bin && Ll.n > 0) {
            const int steps = prop_steps(fo, l, bn->B, n_prop);
            ProfScope prof(ctx, "mark_propagation", s);
            for (int st = 0; st < steps; ++st) {
                hipLaunchKernelGGL(k_prop_spread<D>, dim3(grid_for(Ll.n * (D == 3 ? 26 : 8))), dim3(256), 0, s,
                                   Ll.keys, Ll.n, pm[l], l, fo->roots[0], fo->roots[1], fo->roots[2]);
                hipLaunchKernelGGL(k_prop_commit, dim3(grid_for(Ll.n)), dim3(256), 0, s, pm[l], Ll.n);
            }
        }
        // (ii) balance ripple, level l down to 1
        for (int m = l; m >= 1; --m) {
            if (fo->lev[m].n == 0) continue;
            ProfScope prof(ctx, "balance_ripple", s);
            hipLaunchKernelGGL(k_ripple<D>, dim3(grid_for(fo->lev[m].n * (D == 3 ? 26 : 8))), dim3(256), 0, s,
                               fo->lev[m].keys,
                               fo->lev[m].n, pm[m], m, fo->lev[m - 1].keys, fo->lev[m - 1].n, fo->lev[m - 1].leaf,
                               pm[m - 1], fo->roots[0], fo->roots[1], fo->roots[2], err);
        }
        // (iii) children: count marks per level, then merge level by level
        uint32_t *pos[kMaxLevels + 1] = {};
        uint32_t nmark[kMaxLevels + 2] = {};
        {
            const uint8_t *ins[kMaxLevels + 1];
            int64_t ns[kMaxLevels + 1];
            for (int m = 0; m <= l; ++m) {
                AGAL_TRY(pass.get(&pos[m], (size_t)fo->lev[m].n + 1));
                ins[m] = pm[m];
                ns[m] = fo->lev[m].n;
            }
            // marks per level and the balance error word, back through mapped host memory
            AGAL_TRY(scan_flags_u8_multi(ctx, ins, pos, ns, l + 1, err, nmark, s, scan_status));
        }
        if (nmark[l + 1] != 0) return fail(AGAL_ESTATE, "agal_near_wall_refine: forest lost 2:1 balance");
        // every parent level with marks at once: the new child levels are fresh
        // arrays, and a level that is both a parent (m) and a child (of m - 1)
        // has its leaf and mark bytes set by the first launch before the second
        // copies them
        GrowArgs ga{};
        ga.D = D;
        agal::Level Nl[kMaxLevels + 1];
        int segm[kMaxLevels + 1];
        for (int m = l; m >= 0; --m) {
            const int64_t c = nmark[m];
            agal::Level &P = fo->lev[m];
            agal::Level &C = fo->lev[m + 1];
            if (c == 0) {
                if (m + 1 == l + 1 && C.keys == nullptr) {
                    // no child level yet: an empty one keeps views valid
                    AGAL_TRY(dev_alloc(mem, &C.keys, 1, s));
                    AGAL_TRY(dev_alloc(mem, &C.leaf, 1, s));
                    AGAL_TRY(dev_alloc(mem, &C.mark, 1, s));
                    C.n = 0;
                }
                continue;
            }
            GrowSeg &gs = ga.seg[ga.nseg];
            segm[ga.nseg] = m;
            agal::Level &N = Nl[ga.nseg];
            ++ga.nseg;
            AGAL_TRY(pass.get(&gs.mk, (size_t)c));
            N.n = C.n + (c << D);
            AGAL_TRY(dev_alloc(mem, &N.keys, (size_t)N.n, s));
            AGAL_TRY(dev_alloc(mem, &N.leaf, (size_t)N.n, s));
            AGAL_TRY(dev_alloc(mem, &N.mark, (size_t)N.n, s));
            if (C.cf) AGAL_TRY(dev_alloc(mem, &N.cf, (size_t)N.n * CELLS, s));
            gs.pkeys = P.keys;
            gs.pm = pm[m];
            gs.pos = pos[m];
            gs.pleaf = P.leaf;
            gs.pmark = P.mark;
            gs.pn = P.n;
            gs.c = c;
            gs.ckeys = C.keys;
            gs.cleaf = C.leaf;
            gs.cmark = C.mark;
            gs.ccf = C.cf;
            gs.cn = C.n;
            gs.nkeys = N.keys;
            gs.nleaf = N.leaf;
            gs.nmark = N.mark;
            gs.ncf = N.cf;
        }
        if (ga.nseg > 0) {
            for (int k = 0; k < ga.nseg; ++k) {
                ga.pre_p[k + 1] = ga.pre_p[k] + ga.seg[k].pn;
                ga.pre_g[k + 1] = ga.pre_g[k] + ga.seg[k].cn + (ga.seg[k].c << D);
            }
            ProfScope prof(ctx, "child_gen", s);
            hipLaunchKernelGGL(k_mark_parents_all, dim3(grid_for(ga.pre_p[ga.nseg])), dim3(256), 0, s, ga);
            hipLaunchKernelGGL(k_grow_all<CELLS>, dim3(grid_for(ga.pre_g[ga.nseg])), dim3(256), 0, s, ga);
        }
        for (int k = 0; k < ga.nseg; ++k) {
            agal::Level &C = fo->lev[segm[k] + 1];
            dev_free(mem, C.keys, s);
            dev_free(mem, C.leaf, s);
            dev_free(mem, C.mark, s);
            dev_free(mem, C.cf, s);
            C = Nl[k];
        }
        AGAL_TRY_HIP(hipGetLastError());
    }
    return AGAL_OK;
}

}  // namespace
}  // namespace agal

using namespace agal;

extern "C" {

static agal_status near_wall_refine(agal_geom g, agal_bins b, const agal_forest_desc *desc, void *stream,
                                    agal_forest *out, bool own_bin, int n_prop) {
    if (!g || !b || !desc || !out) return fail(AGAL_EINVAL, "agal_near_wall_refine: NULL argument");
    if (b->geom_id != g->id) return fail(AGAL_ESTATE, "agal_near_wall_refine: bins were built from another geometry");
    if (b->discrete && !own_bin)
        return fail(AGAL_EINVAL, "agal_near_wall_refine: the box test needs bins by bounding box (sampled-point bins "
                                 "can miss a face that crosses a bin between its points); use the own-bin form");
    const int D = desc->dim;
    if (D != g->dim) return fail(AGAL_EINVAL, "agal_near_wall_refine: desc->dim %d != geometry dim %d", D, g->dim);
    if (desc->n_levels < 0 || desc->n_levels > kMaxLevels)
        return fail(AGAL_EINVAL, "agal_near_wall_refine: n_levels must be in [0, %d]", kMaxLevels);
    if (desc->n_levels > 0 && !desc->d_spec) return fail(AGAL_EINVAL, "agal_near_wall_refine: d_spec is NULL");
    uint64_t nroots = 1;
    for (int a = 0; a < D; ++a) {
        if (desc->roots[a] < 1) return fail(AGAL_EINVAL, "agal_near_wall_refine: roots must be >= 1");
        if (!(desc->hi[a] > desc->lo[a])) return fail(AGAL_EINVAL, "agal_near_wall_refine: hi must exceed lo");
        nroots *= (uint64_t)desc->roots[a];
    }
    if ((nroots << (D * desc->n_levels)) > ((uint64_t)1 << 32) || nroots > ((uint64_t)1 << 32))
        return fail(AGAL_EINVAL, "agal_near_wall_refine: roots * 2^(D*n_levels) exceeds the 32-bit key space");
    for (int l = 0; l < desc->n_levels; ++l)
        if (!(desc->d_spec[l] >= 0.0f) || !std::isfinite(desc->d_spec[l]))
            return fail(AGAL_EINVAL, "agal_near_wall_refine: d_spec[%d] must be finite and >= 0", l);

    auto *fo = new (std::nothrow) agal_forest_t();
    if (!fo) return fail(AGAL_ENOMEM, "agal_near_wall_refine: host allocation failed");
    fo->ctx = g->ctx;
    fo->geom_id = g->id;
    fo->stream = (hipStream_t)stream;
    fo->dim = D;
    fo->L = desc->n_levels;
    for (int a = 0; a < 3; ++a) {
        fo->roots[a] = a < D ? desc->roots[a] : 1;
        fo->lo[a] = a < D ? desc->lo[a] : 0.0f;
        fo->hi[a] = a < D ? desc->hi[a] : 1.0f;
    }
    for (int l = 0; l <= fo->L; ++l)
        for (int a = 0; a < 3; ++a) fo->dx[l][a] = (fo->hi[a] - fo->lo[a]) / (float)(4 * fo->roots[a] * (1 << l));
    for (int l = 0; l < fo->L; ++l) fo->d[l] = desc->d_spec[l];
    agal_status st = D == 3 ? refine_impl<3>(g, b, fo, (hipStream_t)stream, own_bin, n_prop)
                            : refine_impl<2>(g, b, fo, (hipStream_t)stream, own_bin, n_prop);
    if (st != AGAL_OK) {
        agal_destroy_forest(fo);
        return st;
    }
    *out = fo;
    return AGAL_OK;
}

agal_status agal_near_wall_refine(agal_geom g, agal_bins b, const agal_forest_desc *desc, void *stream,
                                  agal_forest *out) {
    return near_wall_refine(g, b, desc, stream, out, false, -1);
}

agal_status agal_near_wall_refine_own_bin(agal_geom g, agal_bins b, const agal_forest_desc *desc, int n_prop,
                                          void *stream, agal_forest *out) {
    return near_wall_refine(g, b, desc, stream, out, true, n_prop);
}

agal_status agal_forest_level_view(agal_forest f, int level, const uint32_t **d_keys, const uint8_t **d_leaf,
                                   const uint8_t **d_mark, const uint8_t **d_cell_flag, int64_t *n_blocks) {
    if (!f) return fail(AGAL_EINVAL, "agal_forest_level_view: NULL forest");
    if (level < 0 || level > f->L) return fail(AGAL_EINVAL, "agal_forest_level_view: level %d outside [0, %d]", level, f->L);
    const agal::Level &L = f->lev[level];
    if (d_keys) *d_keys = L.keys;
    if (d_leaf) *d_leaf = L.leaf;
    if (d_mark) *d_mark = L.mark;
    if (d_cell_flag) *d_cell_flag = level < f->L ? L.cf : nullptr;
    if (n_blocks) *n_blocks = L.n;
    return AGAL_OK;
}

agal_status agal_forest_info(agal_forest f, int *dim, int *n_levels) {
    if (!f) return fail(AGAL_EINVAL, "agal_forest_info: NULL forest");
    if (dim) *dim = f->dim;
    if (n_levels) *n_levels = f->L;
    return AGAL_OK;
}

void agal_destroy_forest(agal_forest f) {
    if (!f) return;
    for (int l = 0; l <= kMaxLevels; ++l) {
        dev_free(f->ctx->mem, f->lev[l].keys, f->stream);
        dev_free(f->ctx->mem, f->lev[l].leaf, f->stream);
        dev_free(f->ctx->mem, f->lev[l].mark, f->stream);
        dev_free(f->ctx->mem, f->lev[l].cf, f->stream);
    }
    delete f;
}

}  // extern "C"
