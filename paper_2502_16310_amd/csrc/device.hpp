// Device-side arithmetic shared by the kernels: bin indexing, block keys,
// cell centres, the separating-axis predicate, wave helpers and the
// decoupled look-back used by the ordered compactions.
//
// Every FP32 expression that decides a bin index or a flag is written as a
// fixed sequence of correctly rounded operations; the translation units are
// compiled with -ffp-contract=off (and the pragma below) so none of them is
// fused into an FMA.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

namespace agal {

// Lattice directions (Sec. II-C-1 links follow the discrete velocity set).
// Rest; the axis directions in +/- pairs; the 12 edge directions in +/- pairs;
// the 8 corner directions in +/- pairs.  D3Q19 is the first 19 rows, D3Q27 all
// 27; D2Q9 has its own table.  Direction 2k+1 and 2k+2 are opposite.
constexpr int8_t kDir3[27][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1},
    {1, 0, -1}, {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1},
    {-1, 1, 1}, {1, -1, -1}};
constexpr int8_t kDir2[9][3] = {{0, 0, 0}, {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};

template <int D>
__host__ __device__ constexpr int8_t dir_c(int i, int a) {
    return D == 3 ? kDir3[i][a] : kDir2[i][a];
}

namespace dev {

constexpr int kWave = 64;
constexpr float kEps = 9.5367431640625e-07f;  // 2^-20: margin of every candidate query box

__device__ __forceinline__ float fminf_(float a, float b) { return a < b ? a : b; }
__device__ __forceinline__ float fmaxf_(float a, float b) { return a > b ? a : b; }
__device__ __forceinline__ float fabsf_(float a) { return a < 0.0f ? -a : a; }

// Bin of coordinate x along one axis: floor((x - lo) * s) clamped to [0, B-1];
// clamped in float before the integer conversion.
__device__ __forceinline__ int bin_of(float x, float lo, float s, int B) {
    float t = (x - lo) * s;
    float f = floorf(t);
    if (!(f >= 0.0f)) return 0;   // also a NaN coordinate: stays inside the grid
    if (f > (float)(B - 1)) return B - 1;
    return (int)f;
}

struct BinGrid {
    const uint32_t *off;
    const int32_t *ids;
    float lo[3];
    float s[3];
    int B;
    int64_t F;   // face count: the candidate walkers skip ids outside [0, F)
};

// A value known to be equal on every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Per-face record, one 64-byte (3D) or 32-byte (2D) row per face so that a
// gather of one face touches one cache line:
//   3D: v0 v1 v2 (9 floats), min (3), max (3), 0
//   2D: a b (4 floats), min (2), max (2)
template <int D>
constexpr int kRecFloats = D == 3 ? 16 : 8;

struct Faces {
    const float *coords;  // (D*D) x F
    const float *aabb;    // (2*D) x F
    const float *rec;     // F x kRecFloats<D>
    int64_t F;
};

// The record of face f as kRecFloats<D> / 4 aligned 16-byte loads.
template <int D>
__device__ __forceinline__ void load_rec(const float *rec, int64_t f, float out[kRecFloats<D>]) {
    const float4 *r = reinterpret_cast<const float4 *>(rec) + f * (kRecFloats<D> / 4);
#pragma unroll
    for (int i = 0; i < kRecFloats<D> / 4; ++i) {
        const float4 x = r[i];
        out[4 * i] = x.x;
        out[4 * i + 1] = x.y;
        out[4 * i + 2] = x.z;
        out[4 * i + 3] = x.w;
    }
}

// Block coordinates at `level` from a hierarchical key.
template <int D>
__device__ __forceinline__ void decode_key(uint32_t key, int level, int Rx, int Ry, int c[3]) {
    uint32_t k = key;
    int p0 = 0, p1 = 0, p2 = 0;
    for (int j = 0; j < level; ++j) {
        uint32_t ci = k & ((1u << D) - 1);
        k >>= D;
        p0 |= (int)(ci & 1) << j;
        p1 |= (int)((ci >> 1) & 1) << j;
        if (D == 3) p2 |= (int)((ci >> 2) & 1) << j;
    }
    uint32_t r0 = k % (uint32_t)Rx;
    uint32_t r1 = (k / (uint32_t)Rx) % (uint32_t)Ry;
    uint32_t r2 = k / ((uint32_t)Rx * (uint32_t)Ry);
    c[0] = ((int)r0 << level) | p0;
    c[1] = ((int)r1 << level) | p1;
    c[2] = D == 3 ? (((int)r2 << level) | p2) : 0;
}

// Key of the block at integer coordinates c (level `level`).
template <int D>
__device__ __forceinline__ uint32_t encode_key(const int c[3], int level, int Rx, int Ry) {
    uint32_t r0 = (uint32_t)(c[0] >> level), r1 = (uint32_t)(c[1] >> level);
    uint32_t r2 = D == 3 ? (uint32_t)(c[2] >> level) : 0u;
    uint32_t key = (r2 * (uint32_t)Ry + r1) * (uint32_t)Rx + r0;
    for (int j = level - 1; j >= 0; --j) {
        uint32_t ci = (uint32_t)((c[0] >> j) & 1) | ((uint32_t)((c[1] >> j) & 1) << 1);
        if (D == 3) ci |= (uint32_t)((c[2] >> j) & 1) << 2;
        key = (key << D) | ci;
    }
    return key;
}

// Cell centre coordinate: lo + (float)(2g + 1) * (0.5f * dx).
__device__ __forceinline__ float cell_centre(float lo, int g, float dx) {
    return lo + (float)(2 * g + 1) * (0.5f * dx);
}

// Lower bound of `key` in sorted keys[0..n).
__device__ __forceinline__ int64_t lower_bound_u32(const uint32_t *keys, int64_t n, uint32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Separating-axis predicate: does the closed face meet the closed cube
// [m - h, m + h]^D?  Each axis test is the same rounded expression sequence as
// the definition (separated only on a strict '>'); axes are visited cheapest
// first, which cannot change an OR of independent tests.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool sep3(float p0, float p1, float p2, float r) {
    float mn = fminf_(fminf_(p0, p1), p2);
    float mx = fmaxf_(fmaxf_(p0, p1), p2);
    return (mn > r) || (mx < -r);
}

__device__ __forceinline__ bool sat_triangle(const float v[9], const float m[3], float h) {
    float A0 = v[0] - m[0], A1 = v[1] - m[1], A2 = v[2] - m[2];
    float B0 = v[3] - m[0], B1 = v[4] - m[1], B2 = v[5] - m[2];
    float C0 = v[6] - m[0], C1 = v[7] - m[1], C2 = v[8] - m[2];
    if (sep3(A0, B0, C0, h) || sep3(A1, B1, C1, h) || sep3(A2, B2, C2, h)) return false;
    float E00 = B0 - A0, E01 = B1 - A1, E02 = B2 - A2;
    float E10 = C0 - B0, E11 = C1 - B1, E12 = C2 - B2;
    float E20 = A0 - C0, E21 = A1 - C1, E22 = A2 - C2;
    float N0 = E01 * E12 - E02 * E11;
    float N1 = E02 * E10 - E00 * E12;
    float N2 = E00 * E11 - E01 * E10;
    float s = (N0 * A0 + N1 * A1) + N2 * A2;
    float r = h * ((fabsf_(N0) + fabsf_(N1)) + fabsf_(N2));
    if (s > r || s < -r) return false;
    // e_x x E = (0, -E_z, E_y): components on (y, z)
    // e_y x E = (E_z, 0, -E_x): components on (x, z)
    // e_z x E = (-E_y, E_x, 0): components on (x, y)
#define AGAL_EDGE_AXES(e0, e1, e2)                                                             \
    {                                                                                          \
        float au = -(e2), av = (e1);                                                           \
        float rr = h * (fabsf_(au) + fabsf_(av));                                              \
        if (sep3(au * A1 + av * A2, au * B1 + av * B2, au * C1 + av * C2, rr)) return false;   \
    }                                                                                          \
    {                                                                                          \
        float au = (e2), av = -(e0);                                                           \
        float rr = h * (fabsf_(au) + fabsf_(av));                                              \
        if (sep3(au * A0 + av * A2, au * B0 + av * B2, au * C0 + av * C2, rr)) return false;   \
    }                                                                                          \
    {                                                                                          \
        float au = -(e1), av = (e0);                                                           \
        float rr = h * (fabsf_(au) + fabsf_(av));                                              \
        if (sep3(au * A0 + av * A1, au * B0 + av * B1, au * C0 + av * C1, rr)) return false;   \
    }
    AGAL_EDGE_AXES(E00, E01, E02)
    AGAL_EDGE_AXES(E10, E11, E12)
    AGAL_EDGE_AXES(E20, E21, E22)
#undef AGAL_EDGE_AXES
    return true;
}

__device__ __forceinline__ bool sat_segment(const float v[4], const float m[2], float h) {
    float A0 = v[0] - m[0], A1 = v[1] - m[1];
    float B0 = v[2] - m[0], B1 = v[3] - m[1];
    if (fminf_(A0, B0) > h || fmaxf_(A0, B0) < -h) return false;
    if (fminf_(A1, B1) > h || fmaxf_(A1, B1) < -h) return false;
    float Nx = -(B1 - A1);
    float Ny = B0 - A0;
    float pA = Nx * A0 + Ny * A1;
    float pB = Nx * B0 + Ny * B1;
    float r = h * (fabsf_(Nx) + fabsf_(Ny));
    if (fminf_(pA, pB) > r || fmaxf_(pA, pB) < -r) return false;
    return true;
}


// Euclidean near test of the paper's face detection (Sec. II-C-2, Algorithm
// 1): is the point p within distance R of the closed face?  Decided in FP32
// as one fixed sequence of rounded operations, without divisions (a squared
// distance c / m is compared as c <= R^2 m):
//   R2 = R * R; for each closed edge [a, b] (2D: the segment; 3D: the three
//   edges (v0,v1), (v1,v2), (v2,v0)), with w = p - a, e = b - a, we = w.e:
//     we <= 0   -> near when w.w <= R2 (the nearest point is a);
//     we >= e.e -> near when u.u <= R2, u = p - b (the nearest point is b);
//     otherwise -> near when |e x w|^2 <= R2 (e.e) (2D: (e0 w1 - e1 w0)^2);
//   3D, the face itself: n = (v1 - v0) x (v2 - v0); when n.n > 0 and p
//   projects inside (((v_{k+1} - v_k) x (p - v_k)) . n >= 0 for all three
//   edges), near when ((p - v0) . n)^2 <= R2 (n.n).
// Dot products are (x0 y0 + x1 y1) + x2 y2, cross products
// (a1 b2 - a2 b1, a2 b0 - a0 b2, a0 b1 - a1 b0).
__device__ __forceinline__ float dot3_(const float *a, const float *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
__device__ __forceinline__ void cross3_(const float *a, const float *b, float *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

template <int D>
__device__ __forceinline__ bool edge_near_l2(const float *a, const float *b, const float *p, float R2) {
    float w[3] = {0.0f, 0.0f, 0.0f}, e[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        w[k] = p[k] - a[k];
        e[k] = b[k] - a[k];
    }
    const float we = D == 3 ? dot3_(w, e) : w[0] * e[0] + w[1] * e[1];
    if (we <= 0.0f) return (D == 3 ? dot3_(w, w) : w[0] * w[0] + w[1] * w[1]) <= R2;
    const float ee = D == 3 ? dot3_(e, e) : e[0] * e[0] + e[1] * e[1];
    if (we >= ee) {
        float u[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = p[k] - b[k];
        return (D == 3 ? dot3_(u, u) : u[0] * u[0] + u[1] * u[1]) <= R2;
    }
    float cc;
    if constexpr (D == 3) {
        float c[3];
        cross3_(e, w, c);
        cc = dot3_(c, c);
    } else {
        const float cr = e[0] * w[1] - e[1] * w[0];
        cc = cr * cr;
    }
    return cc <= R2 * ee;
}

template <int D>
__device__ __forceinline__ bool near_l2(const float *v, const float *p, float R) {
    const float R2 = R * R;
    if constexpr (D == 2) {
        return edge_near_l2<2>(v, v + 2, p, R2);
    } else {
        if (edge_near_l2<3>(v, v + 3, p, R2) || edge_near_l2<3>(v + 3, v + 6, p, R2) ||
            edge_near_l2<3>(v + 6, v, p, R2))
            return true;
        float e1[3], e2[3], n[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            e1[a] = v[3 + a] - v[a];
            e2[a] = v[6 + a] - v[a];
        }
        cross3_(e1, e2, n);
        const float nn = dot3_(n, n);
        if (!(nn > 0.0f)) return false;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float *a = v + 3 * k, *b = v + 3 * ((k + 1) % 3);
            float e[3], w[3], c[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                e[j] = b[j] - a[j];
                w[j] = p[j] - a[j];
            }
            cross3_(e, w, c);
            if (!(dot3_(c, n) >= 0.0f)) return false;
        }
        float w0[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) w0[j] = p[j] - v[j];
        const float hh = dot3_(w0, n);
        return hh * hh <= R2 * nn;
    }
}
// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Completion signal to the host through mapped host memory.  One thread
// calls it once it has written everything the host is to read (mapped host
// words): a system-scope fence orders those writes before the store of seq
// into *word, so a host that reads seq sees them.  The rest of the kernel's
// output is only read by later work on the same stream, which stream order
// covers.  word == null: no signal.  (A fence per workgroup would write the
// L2 back once per workgroup: 0.3 ms for a 327,680-face import.)
__device__ __forceinline__ void publish_host(uint32_t *word, uint32_t seq) {
    if (!word) return;
    __threadfence_system();
    __hip_atomic_store(word, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// For a signal that needs n arrivals (each from one thread, after its own
// host writes): counts the caller in *done (a device word that is zero before
// and left zero after) and returns true to the last arrival, which then
// publishes.
__device__ __forceinline__ bool arrive_last(uint32_t *done, uint32_t n) {
    __threadfence_system();
    if (__hip_atomic_fetch_add(done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM) != n - 1u) return false;
    __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return true;
}

// Orders the LDS accesses of the lanes of one wave before and after it (data
// passed between lanes of a wave through LDS).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Decoupled look-back (single-pass ordered prefix over tiles).  Tiles take
// their index from a ticket counter in launch order, publish their aggregate,
// then sum predecessors' values until one has published its inclusive
// prefix.  Status word: bits 32..33 flag (1 aggregate, 2 inclusive), low 32
// bits the value.  All status traffic is agent-scope atomics, so tiles on
// different XCDs observe each other.
// ---------------------------------------------------------------------------
constexpr uint64_t kAgg = 1ull << 32;
constexpr uint64_t kInc = 2ull << 32;

__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_load(uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by one full wave; returns the exclusive prefix of `tile` (uniform).
__device__ __forceinline__ uint32_t lookback_wave(uint64_t *status, uint32_t tile, uint32_t aggregate) {
    const int lane = lane_id();
    if (tile == 0) {
        if (lane == 0) status_store(&status[0], kInc | aggregate);
        return 0u;
    }
    if (lane == 0) status_store(&status[tile], kAgg | aggregate);
    uint32_t prefix = 0;
    int64_t base = (int64_t)tile - 1;
    while (true) {
        int64_t j = base - lane;
        uint64_t w = kInc;  // lanes before tile 0 read as an inclusive zero
        if (j >= 0) {
            do {
                w = status_load(&status[j]);
                if ((w >> 32) == 0) __builtin_amdgcn_s_sleep(1);
            } while ((w >> 32) == 0);
        }
        uint64_t inc_mask = __ballot((w >> 32) == 2);
        uint32_t val = (uint32_t)w;
        if (inc_mask) {
            int first = __ffsll((unsigned long long)inc_mask) - 1;  // nearest inclusive predecessor
            uint32_t contrib = lane <= first ? val : 0u;
            prefix += wave_sum(contrib);
            break;
        }
        prefix += wave_sum(val);
        base -= kWave;
    }
    if (lane == 0) status_store(&status[tile], kInc | (prefix + aggregate));
    return prefix;
}

}  // namespace dev
}  // namespace agal
