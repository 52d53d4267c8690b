// The paper's own binning (Sec. II-C-3 and its discretization figure): each
// face is sampled at points whose number grows with its size and goes to every
// bin that holds one of them.  An edge a -> b, e = b - a, is cut into 2^k equal
// pieces, k the least integer >= 0 with max_a |e_a| <= spacing * 2^k (k at most
// kDiscKMax); its points are a + e * (j 2^-k), j = 0 .. 2^k (one FP32 product
// and one FP32 sum per component, exact parameters).  A triangle (a, b, c)
// takes the points q_j of its edge a -> b and samples every segment q_j -> c
// the same way; a 2D face is its edge.  Points go to bins by the box binning's
// index function, so the bins of a face are those of its points, found in
// FP32 by the same expressions on every device.
//
// Two forms, one result (per bin, ascending face ids):
//  * pairs (bin_fraction 0): one thread per face collects its distinct bins
//    in a 64-bit mask over its bin range (the bounding-box bins widened by one
//    per side, which every rounded point stays inside); faces with larger
//    ranges are listed and taken by a workgroup each, with an LDS bit mask
//    over chunks of the range.  Count, scan, scatter with combined atomics,
//    then the canonical order as for the box binning (bins too large for LDS
//    rebuilt by an ordered sweep that resamples the candidate faces);
//  * the paper's bin-fraction form (bin_fraction B_f >= 1): the bins are
//    taken B_n = ceil(B^D / B_f) at a time; an indicator array of B_n x F
//    words (bin-major, -1 = absent) is filled by one thread per face, then
//    each bin's row is counted and compacted in face order into the output,
//    whose length starts at ten entries per face, as in the paper, and is
//    redone at the exact length if that proves short.
#include <algorithm>
#include <cmath>

#include "agal_internal.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace agal {
namespace {

using namespace kern;

constexpr int kDiscKMax = 12;
constexpr int kDiscBigThreads = 256;
constexpr int kDiscChunkWords = 1024;                 // LDS bit mask of the big-face path: 32768 bins per chunk
constexpr int kDiscChunkBins = kDiscChunkWords * 32;
constexpr int kRowThreads = 256;

struct DiscGrid {
    dev::BinGrid g;
    float spacing;
};

template <int D>
__device__ __forceinline__ int disc_k(const float e[3], float spacing) {
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const float m = fabsf(e[a]);
        s = m > s ? m : s;
    }
    int k = 0;
    while (k < kDiscKMax && !(s <= ldexpf(spacing, k))) ++k;
    return k;
}

// Every sample point of the face with corners v (D x D floats); visit(p)
// returns false to stop early.
template <int D, class Visit>
__device__ __forceinline__ void disc_points(const float *v, float spacing, Visit &&visit) {
    float e[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < D; ++a) e[a] = v[D + a] - v[a];
    const int k1 = disc_k<D>(e, spacing);
    const int n1 = 1 << k1;
    for (int j = 0; j <= n1; ++j) {
        const float t = ldexpf((float)j, -k1);
        float q[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int a = 0; a < D; ++a) q[a] = v[a] + e[a] * t;
        if constexpr (D == 3) {
            const float g[3] = {v[6] - q[0], v[7] - q[1], v[8] - q[2]};
            const int k2 = disc_k<3>(g, spacing);
            const int n2 = 1 << k2;
            for (int i = 0; i <= n2; ++i) {
                const float u = ldexpf((float)i, -k2);
                const float p[3] = {q[0] + g[0] * u, q[1] + g[1] * u, q[2] + g[2] * u};
                if (!visit(p)) return;
            }
        } else {
            if (!visit(q)) return;
        }
    }
}

// The face's bin range: its bounding-box bins widened by one per side.
template <int D>
__device__ __forceinline__ void disc_range(const float *r, const dev::BinGrid &g, int lo[3], int n[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = 0;
        n[a] = 1;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int l = max(dev::bin_of(r[D * D + a], g.lo[a], g.s[a], g.B) - 1, 0);
        const int h = min(dev::bin_of(r[D * D + D + a], g.lo[a], g.s[a], g.B) + 1, g.B - 1);
        lo[a] = l;
        n[a] = h - l + 1;
    }
}

template <int D>
__device__ __forceinline__ int64_t point_bin(const float p[3], const dev::BinGrid &g, int ix[3]) {
    ix[0] = ix[1] = ix[2] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) ix[a] = dev::bin_of(p[a], g.lo[a], g.s[a], g.B);
    return ((int64_t)ix[2] * g.B + ix[1]) * g.B + ix[0];
}

// ---- pairs form --------------------------------------------------------------
// One thread per face: the distinct bins of its points in a 64-bit mask over
// its range; a face whose range holds more than 64 bins (or, should rounding
// ever carry a point past it, any face with such a point) goes to the big
// list in the count pass and is left to k_disc_big in both passes.
template <int D, bool kScatter>
__global__ void k_disc_small(const float *rec, int64_t F, DiscGrid G, uint32_t *count, const uint32_t *off,
                             uint32_t *cursor, int32_t *ids, uint32_t *big_list, uint32_t *nbig) {
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
        float r[dev::kRecFloats<D>];
        dev::load_rec<D>(rec, f, r);
        int lo[3], n[3];
        disc_range<D>(r, G.g, lo, n);
        if ((int64_t)n[0] * n[1] * n[2] > 64) {
            if (!kScatter) big_list[atomicAdd(nbig, 1u)] = (uint32_t)f;
            continue;
        }
        uint64_t mask = 0;
        bool outside = false;   // a point beyond the widened box range: the face takes the workgroup path
        disc_points<D>(r, G.spacing, [&](const float p[3]) {
            int ix[3];
            (void)point_bin<D>(p, G.g, ix);
#pragma unroll
            for (int a = 0; a < 3; ++a) outside |= ix[a] < lo[a] || ix[a] >= lo[a] + n[a];
            if (outside) return false;
            const int l = ((ix[2] - lo[2]) * n[1] + (ix[1] - lo[1])) * n[0] + (ix[0] - lo[0]);
            mask |= 1ull << l;
            return true;
        });
        if (outside) {
            if (!kScatter) big_list[atomicAdd(nbig, 1u)] = (uint32_t)f;
            continue;
        }
        while (mask) {
            const int l = __builtin_ctzll(mask);
            mask &= mask - 1ull;
            const int x = lo[0] + l % n[0], y = lo[1] + (l / n[0]) % n[1], z = lo[2] + l / (n[0] * n[1]);
            const int64_t b = ((int64_t)z * G.g.B + y) * G.g.B + x;
            if constexpr (kScatter) ids[off[b] + add_one_combined(cursor + b)] = (int32_t)f;
            else (void)add_one_combined(count + b);
        }
    }
}

// Every point of the face's fans that thread `t` of `nt` samples (edge points
// t, t + nt, ..., each with its whole segment to the opposite vertex).
template <int D, class Visit>
__device__ __forceinline__ void disc_points_strided(const float *r, float spacing, int t, int nt, Visit &&visit) {
    float e[3] = {0.0f, 0.0f, 0.0f};
    for (int a = 0; a < D; ++a) e[a] = r[D + a] - r[a];
    const int k1 = disc_k<D>(e, spacing);
    const int n1 = 1 << k1;
    for (int j = t; j <= n1; j += nt) {
        const float tj = ldexpf((float)j, -k1);
        float q[3] = {0.0f, 0.0f, 0.0f};
        for (int a = 0; a < D; ++a) q[a] = r[a] + e[a] * tj;
        if constexpr (D == 3) {
            const float g[3] = {r[6] - q[0], r[7] - q[1], r[8] - q[2]};
            const int k2 = disc_k<3>(g, spacing);
            const int n2 = 1 << k2;
            for (int i = 0; i <= n2; ++i) {
                const float u = ldexpf((float)i, -k2);
                const float p[3] = {q[0] + g[0] * u, q[1] + g[1] * u, q[2] + g[2] * u};
                visit(p);
            }
        } else {
            visit(q);
        }
    }
}

// One workgroup per listed face: the bin range of its points (a first sweep),
// then the range in chunks of kDiscChunkBins bins with an LDS bit per bin; the
// threads share the face's edge points (each samples its own fan segments),
// then walk the set bits.
template <int D, bool kScatter>
__global__ __launch_bounds__(kDiscBigThreads) void k_disc_big(const float *rec, DiscGrid G, const uint32_t *big_list,
                                                              const uint32_t *nbig, uint32_t *count,
                                                              const uint32_t *off, uint32_t *cursor, int32_t *ids) {
    __shared__ uint32_t s_mask[kDiscChunkWords];
    __shared__ int s_lo[3], s_hi[3];
    const uint32_t nf = *nbig;
    for (uint32_t bi = blockIdx.x; bi < nf; bi += gridDim.x) {
        const int64_t f = big_list[bi];
        float r[dev::kRecFloats<D>];
        dev::load_rec<D>(rec, f, r);
        if (threadIdx.x < 3) {
            s_lo[threadIdx.x] = threadIdx.x < D ? G.g.B : 0;
            s_hi[threadIdx.x] = 0;
        }
        __syncthreads();
        {
            int mn[3] = {G.g.B, G.g.B, G.g.B}, mx[3] = {-1, -1, -1};
            disc_points_strided<D>(r, G.spacing, threadIdx.x, kDiscBigThreads, [&](const float p[3]) {
                int ix[3];
                (void)point_bin<D>(p, G.g, ix);
                for (int a = 0; a < D; ++a) {
                    mn[a] = min(mn[a], ix[a]);
                    mx[a] = max(mx[a], ix[a]);
                }
            });
            for (int a = 0; a < D; ++a)
                if (mx[a] >= 0) {
                    atomicMin(&s_lo[a], mn[a]);
                    atomicMax(&s_hi[a], mx[a]);
                }
        }
        __syncthreads();
        const int lo[3] = {s_lo[0], s_lo[1], s_lo[2]};
        const int n[3] = {s_hi[0] - s_lo[0] + 1, s_hi[1] - s_lo[1] + 1, s_hi[2] - s_lo[2] + 1};
        const int64_t nr = (int64_t)n[0] * n[1] * n[2];
        __syncthreads();   // every thread has its range before s_lo / s_hi are reset for the next face
        for (int64_t c0 = 0; c0 < nr; c0 += kDiscChunkBins) {
            for (int w = threadIdx.x; w < kDiscChunkWords; w += kDiscBigThreads) s_mask[w] = 0u;
            __syncthreads();
            disc_points_strided<D>(r, G.spacing, threadIdx.x, kDiscBigThreads, [&](const float p[3]) {
                int ix[3];
                (void)point_bin<D>(p, G.g, ix);
                const int64_t l = ((int64_t)(ix[2] - lo[2]) * n[1] + (ix[1] - lo[1])) * n[0] + (ix[0] - lo[0]);
                if (l >= c0 && l < c0 + kDiscChunkBins) atomicOr(&s_mask[(l - c0) >> 5], 1u << ((l - c0) & 31));
            });
            __syncthreads();
            for (int w = threadIdx.x; w < kDiscChunkWords; w += kDiscBigThreads) {
                uint32_t m = s_mask[w];
                while (m) {
                    const int bit = __builtin_ctz(m);
                    m &= m - 1u;
                    const int64_t l = c0 + 32 * w + bit;
                    const int x = lo[0] + (int)(l % n[0]), y = lo[1] + (int)((l / n[0]) % n[1]);
                    const int z = lo[2] + (int)(l / ((int64_t)n[0] * n[1]));
                    const int64_t b = ((int64_t)z * G.g.B + y) * G.g.B + x;
                    if constexpr (kScatter) ids[off[b] + atomicAdd(cursor + b, 1u)] = (int32_t)f;
                    else atomicAdd(count + b, 1u);
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(64) void k_disc_canon_small(int32_t *ids, const uint32_t *off, int64_t nb,
                                                         uint32_t *med_list, uint32_t *big_list, uint32_t *counts) {
    bin_canon_group(ids, off, nb, (int64_t)blockIdx.x * dev::kWave, med_list, big_list, counts, 0u);
}

__global__ __launch_bounds__(kMedThreads) void k_disc_canon_medium(int32_t *ids, const uint32_t *off,
                                                                   const uint32_t *med_list, const uint32_t *counts) {
    const uint32_t nmed = counts[0];
    for (uint32_t i = blockIdx.x; i < nmed; i += gridDim.x) bin_canon_medium(ids, off, med_list[i]);
}

// Bins with more than kCanonCap ids: rewritten by an ordered sweep over all
// faces, each resampled until a point lands in the bin (such bins only occur
// when the bins are few and large).
template <int D>
__global__ __launch_bounds__(kBigThreads) void k_disc_canon_big(const float *rec, int64_t F, DiscGrid G,
                                                                const uint32_t *off, int32_t *ids,
                                                                const uint32_t *big_list, const uint32_t *counts) {
    __shared__ uint32_t s_wsum[kBigThreads / dev::kWave];
    const uint32_t nbig = counts[1];
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x % dev::kWave;
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const int64_t b = big_list[bi];
        uint32_t run = off[b];
        for (int64_t f0 = 0; f0 < F; f0 += kBigThreads) {
            const int64_t f = f0 + threadIdx.x;
            uint32_t mem = 0;
            if (f < F) {
                float r[dev::kRecFloats<D>];
                dev::load_rec<D>(rec, f, r);
                disc_points<D>(r, G.spacing, [&](const float p[3]) {
                    int ix[3];
                    if (point_bin<D>(p, G.g, ix) == b) mem = 1u;
                    return mem == 0u;
                });
            }
            const uint32_t incl = dev::wave_inclusive_sum(mem);
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

// ---- the paper's bin-fraction form --------------------------------------------
// Indicator rows of bins c0 .. c0 + bn - 1: ind[(b - c0) * F + f] = f when a
// point of face f lies in bin b (the rows start at -1).
template <int D>
__global__ void k_disc_mark(const float *rec, int64_t F, DiscGrid G, int64_t c0, int64_t bn, int32_t *ind) {
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
        float r[dev::kRecFloats<D>];
        dev::load_rec<D>(rec, f, r);
        disc_points<D>(r, G.spacing, [&](const float p[3]) {
            int ix[3];
            const int64_t b = point_bin<D>(p, G.g, ix);
            if (b >= c0 && b < c0 + bn) ind[(b - c0) * F + f] = (int32_t)f;
            return true;
        });
    }
}

// Entries of each indicator row (one workgroup per row).
__global__ __launch_bounds__(kRowThreads) void k_disc_rows(const int32_t *ind, int64_t F, int64_t bn,
                                                           uint32_t *count) {
    __shared__ uint32_t s_acc;
    for (int64_t row = blockIdx.x; row < bn; row += gridDim.x) {
        if (threadIdx.x == 0) s_acc = 0u;
        __syncthreads();
        uint32_t c = 0;
        const int32_t *x = ind + row * F;
        for (int64_t f = threadIdx.x; f < F; f += kRowThreads) c += x[f] >= 0 ? 1u : 0u;
        for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, dev::kWave);
        if (dev::lane_id() == 0 && c) atomicAdd(&s_acc, c);
        __syncthreads();
        if (threadIdx.x == 0) count[row] = s_acc;
        __syncthreads();
    }
}

// Each row compacted in face order to ids[off[row] ..) (writes at or past cap
// are dropped; the caller redoes the binning at the exact length).
__global__ __launch_bounds__(kRowThreads) void k_disc_copy(const int32_t *ind, int64_t F, int64_t bn,
                                                           const uint32_t *off, int32_t *ids, uint32_t cap) {
    __shared__ uint32_t s_wsum[kRowThreads / dev::kWave];
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x % dev::kWave;
    for (int64_t row = blockIdx.x; row < bn; row += gridDim.x) {
        const int32_t *x = ind + row * F;
        uint32_t run = off[row];
        for (int64_t f0 = 0; f0 < F; f0 += kRowThreads) {
            const int64_t f = f0 + threadIdx.x;
            const int32_t v = f < F ? x[f] : -1;
            const uint32_t mem = v >= 0 ? 1u : 0u;
            const uint32_t incl = dev::wave_inclusive_sum(mem);
            if (lane == dev::kWave - 1) s_wsum[w] = incl;
            __syncthreads();
            uint32_t pre = 0, tot = 0;
            for (int j = 0; j < kRowThreads / dev::kWave; ++j) {
                if (j < w) pre += s_wsum[j];
                tot += s_wsum[j];
            }
            const uint32_t pos = run + pre + incl - 1;
            if (mem && pos < cap) ids[pos] = v;
            run += tot;
            __syncthreads();
        }
    }
}

unsigned grid_of(int64_t n, int threads = 256, int64_t cap = 8192) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, cap));
}

template <int D>
agal_status disc_pairs(agal_geom g, agal_bins bn, const DiscGrid &G, hipStream_t s) {
    agal_context ctx = g->ctx;
    const int64_t nb = bn->nb, F = g->F;
    uint32_t *count = nullptr, *cursor = nullptr, *big_faces = nullptr, *med = nullptr, *big = nullptr;
    auto done = [&](agal_status st) {
        dev_free(ctx->mem, count, s);
        dev_free(ctx->mem, big_faces, s);
        dev_free(ctx->mem, med, s);
        dev_free(ctx->mem, big, s);
        return st;
    };
    // count + cursor (2 nb), then: big-face count, canon list counts (2)
    AGAL_TRY(dev_alloc(ctx->mem, &count, (size_t)2 * nb + 4, s));
    cursor = count + nb;
    uint32_t *nbig = count + 2 * nb, *lists = count + 2 * nb + 1;
    fill_u32(count, 0u, 2 * nb + 4, s);
    agal_status st = dev_alloc(ctx->mem, &big_faces, (size_t)std::max<int64_t>(F, 1), s);
    if (st != AGAL_OK) return done(st);
    const unsigned big_grid = (unsigned)std::min<int64_t>(std::max<int64_t>(F, 1), 2048);
    {
        ProfScope prof(ctx, "bin_disc_count", s);
        hipLaunchKernelGGL((k_disc_small<D, false>), dim3(grid_of(F)), dim3(256), 0, s, g->rec, F, G, count, nullptr,
                           nullptr, nullptr, big_faces, nbig);
        hipLaunchKernelGGL((k_disc_big<D, false>), dim3(big_grid), dim3(kDiscBigThreads), 0, s, g->rec, G, big_faces, nbig,
                           count, nullptr, nullptr, nullptr);
    }
    AGAL_TRY_HIP(hipGetLastError());
    uint32_t P = 0;
    st = scan_u32_total(ctx, count, bn->off, nb, nullptr, &P, s);
    if (st != AGAL_OK) return done(st);
    bn->P = P;
    st = dev_alloc(ctx->mem, &bn->ids, (size_t)std::max<uint32_t>(P, 1u), s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &med, (size_t)nb, s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &big, (size_t)P / kCanonCap + 1, s);
    if (st != AGAL_OK) return done(st);
    {
        ProfScope prof(ctx, "bin_disc_scatter", s);
        hipLaunchKernelGGL((k_disc_small<D, true>), dim3(grid_of(F)), dim3(256), 0, s, g->rec, F, G, nullptr, bn->off,
                           cursor, bn->ids, big_faces, nbig);
        hipLaunchKernelGGL((k_disc_big<D, true>), dim3(big_grid), dim3(kDiscBigThreads), 0, s, g->rec, G, big_faces, nbig,
                           nullptr, bn->off, cursor, bn->ids);
    }
    {
        ProfScope prof(ctx, "bin_canon", s);
        hipLaunchKernelGGL(k_disc_canon_small, dim3((unsigned)((nb + dev::kWave - 1) / dev::kWave)), dim3(dev::kWave),
                           0, s, bn->ids, bn->off, nb, med, big, lists);
        hipLaunchKernelGGL(k_disc_canon_medium, dim3((unsigned)std::min<int64_t>(nb, 8192)), dim3(kMedThreads), 0, s,
                           bn->ids, bn->off, med, lists);
        hipLaunchKernelGGL((k_disc_canon_big<D>), dim3((unsigned)std::min<int64_t>((int64_t)P / kCanonCap + 1, 256)),
                           dim3(kBigThreads), 0, s, g->rec, F, G, bn->off, bn->ids, big, lists);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return done(fail(AGAL_EHIP, "agal_bin_faces_discrete: launch failed: %s", hipGetErrorString(e)));
    return done(AGAL_OK);
}

// Largest indicator array of the bin-fraction form.
constexpr int64_t kMaxIndicatorBytes = int64_t(32) << 30;

template <int D>
agal_status disc_fractions(agal_geom g, agal_bins bn, const DiscGrid &G, int64_t bf, hipStream_t s) {
    agal_context ctx = g->ctx;
    const int64_t nb = bn->nb, F = g->F;
    const int64_t bnum = (nb + bf - 1) / bf;   // bins per fraction
    if (bnum * std::max<int64_t>(F, 1) * 4 > kMaxIndicatorBytes)
        return fail(AGAL_ECAPACITY,
                    "agal_bin_faces_discrete: %lld bins per fraction x %lld faces exceed the %lld GiB indicator "
                    "limit; raise bin_fraction",
                    (long long)bnum, (long long)F, (long long)(kMaxIndicatorBytes >> 30));
    int32_t *ind = nullptr;
    uint32_t *count = nullptr;
    auto done = [&](agal_status st) {
        dev_free(ctx->mem, ind, s);
        dev_free(ctx->mem, count, s);
        return st;
    };
    AGAL_TRY(dev_alloc(ctx->mem, &ind, (size_t)std::max<int64_t>(bnum * F, 1), s));
    agal_status st = dev_alloc(ctx->mem, &count, (size_t)nb, s);
    if (st != AGAL_OK) return done(st);
    int64_t cap = std::min<int64_t>(10 * std::max<int64_t>(F, 1), (int64_t)UINT32_MAX);   // the paper's first guess
    for (int attempt = 0; attempt < 2; ++attempt) {
        dev_free(ctx->mem, bn->ids, s);
        st = dev_alloc(ctx->mem, &bn->ids, (size_t)cap, s);
        if (st != AGAL_OK) return done(st);
        for (int64_t c0 = 0; c0 < nb; c0 += bnum) {
            const int64_t n = std::min<int64_t>(bnum, nb - c0);
            {
                ProfScope prof(ctx, "bin_disc_mark", s);
                fill_u32(reinterpret_cast<uint32_t *>(ind), 0xFFFFFFFFu, n * F, s);
                hipLaunchKernelGGL((k_disc_mark<D>), dim3(grid_of(F)), dim3(256), 0, s, g->rec, F, G, c0, n, ind);
            }
            {
                ProfScope prof(ctx, "bin_disc_rows", s);
                hipLaunchKernelGGL(k_disc_rows, dim3((unsigned)std::min<int64_t>(n, 65536)), dim3(kRowThreads), 0, s,
                                   ind, F, n, count + c0);
            }
            st = scan_u32(ctx, count, bn->off, c0 + n, s);
            if (st != AGAL_OK) return done(st);
            {
                ProfScope prof(ctx, "bin_disc_copy", s);
                hipLaunchKernelGGL(k_disc_copy, dim3((unsigned)std::min<int64_t>(n, 65536)), dim3(kRowThreads), 0, s,
                                   ind, F, n, bn->off + c0, bn->ids, (uint32_t)cap);
            }
            AGAL_TRY_HIP(hipGetLastError());
        }
        uint32_t P = 0;
        AGAL_TRY_HIP(hipMemcpyAsync(&P, bn->off + nb, 4, hipMemcpyDeviceToHost, s));
        AGAL_TRY_HIP(hipStreamSynchronize(s));
        bn->P = P;
        if ((int64_t)P <= cap) return done(AGAL_OK);
        cap = P;   // the first guess was short: once more at the exact length
    }
    return done(fail(AGAL_EHIP, "agal_bin_faces_discrete: entry count changed between passes"));
}

}  // namespace
}  // namespace agal

using namespace agal;

extern "C" {

agal_status agal_bin_faces_discrete(agal_geom g, const float lo[3], const float hi[3], int32_t B, float spacing,
                                    int32_t bin_fraction, void *stream, agal_bins *out) {
    if (!g || !lo || !hi || !out) return fail(AGAL_EINVAL, "agal_bin_faces_discrete: NULL argument");
    if (B < 1) return fail(AGAL_EINVAL, "agal_bin_faces_discrete: B must be >= 1 (got %d)", B);
    if (bin_fraction < 0) return fail(AGAL_EINVAL, "agal_bin_faces_discrete: negative bin_fraction");
    if (std::isnan(spacing)) return fail(AGAL_EINVAL, "agal_bin_faces_discrete: spacing is NaN");
    const int D = g->dim;
    int64_t nb = 1;
    float smin = INFINITY;
    DiscGrid G{};
    for (int a = 0; a < D; ++a) {
        if (!(hi[a] > lo[a])) return fail(AGAL_EINVAL, "agal_bin_faces_discrete: hi must exceed lo on every axis");
        if (nb > ((int64_t)1 << 31) / B) return fail(AGAL_EINVAL, "agal_bin_faces_discrete: B^D exceeds 2^31");
        nb *= B;
        smin = std::min(smin, (hi[a] - lo[a]) / (float)B);
    }
    if (!(spacing > 0.0f)) spacing = 0.5f * smin;   // default: half the smallest bin edge
    if (!std::isfinite(spacing)) return fail(AGAL_EINVAL, "agal_bin_faces_discrete: spacing must be finite");
    G.spacing = spacing;
    hipStream_t s = (hipStream_t)stream;
    agal_context ctx = g->ctx;
    auto *bn = new (std::nothrow) agal_bins_t();
    if (!bn) return fail(AGAL_ENOMEM, "agal_bin_faces_discrete: host allocation failed");
    bn->ctx = ctx;
    bn->geom_id = g->id;
    bn->stream = s;
    bn->dim = D;
    bn->B = B;
    bn->nb = nb;
    bn->discrete = true;
    bn->spacing = spacing;
    G.g.B = B;
    for (int a = 0; a < 3; ++a) {
        bn->lo[a] = a < D ? lo[a] : 0.0f;
        bn->hi[a] = a < D ? hi[a] : 1.0f;
        bn->s[a] = (float)B / (bn->hi[a] - bn->lo[a]);
        G.g.lo[a] = bn->lo[a];
        G.g.s[a] = bn->s[a];
    }
    agal_status st = dev_alloc(ctx->mem, &bn->off, (size_t)nb + 1, s);
    if (st == AGAL_OK) {
        if (bin_fraction == 0)
            st = D == 3 ? disc_pairs<3>(g, bn, G, s) : disc_pairs<2>(g, bn, G, s);
        else
            st = D == 3 ? disc_fractions<3>(g, bn, G, bin_fraction, s) : disc_fractions<2>(g, bn, G, bin_fraction, s);
    }
    if (st != AGAL_OK) {
        agal_destroy_bins(bn);
        return st;
    }
    *out = bn;
    return AGAL_OK;
}

}  // extern "C"
