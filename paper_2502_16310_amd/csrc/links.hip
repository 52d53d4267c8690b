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

namespace agal {
namespace {

constexpr int kLinkCap = 128;  // staged faces per wave

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
    uint32_t *count;       // nodes per block (staging)
    uint64_t *node_key;    // staging: block * 4^D + rank
    float *q;
    int32_t *face;
};

template <int D, int Q>
__global__ __launch_bounds__(64) void k_links(LinkArgs<D, Q> A) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    constexpr int BPW = 64 / CELLS;
    constexpr int NP = (Q - 1) / 2;            // direction pairs
    constexpr int NF = D == 3 ? 18 : 8;        // floats staged per face
    __shared__ float s_f[NF][kLinkCap];
    __shared__ int32_t s_id[kLinkCap];
    __shared__ float s_dir[NP][3];   // D = c * dx of each direction pair's first direction
    const int lane = threadIdx.x;
    if (lane < NP)
        for (int a = 0; a < 3; ++a) s_dir[lane][a] = (float)dir_c<D>(1 + 2 * lane, a) * A.dx[a];
    const int64_t first = (int64_t)blockIdx.x * BPW;
    const int64_t blk = first + lane / CELLS;
    const bool valid = blk < A.n;
    const int cell = lane % CELLS;
    const int64_t F = A.faces.F;

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
    float clo[3], chi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        clo[a] = (o[a] - A.dx[a]) - A.eps[a];
        chi[a] = (o[a] + A.dx[a]) + A.eps[a];
    }

    float best_t[Q - 1];
    int32_t best_f[Q - 1];
#pragma unroll
    for (int i = 0; i < Q - 1; ++i) {
        best_t[i] = 2.0f;
        best_f[i] = -1;
    }

    // t is decided in FP64 and kept rounded to FP32; equal FP32 values go to the
    // lower face id (both faces are then hits at the same q).
    auto consider = [&](int i, double t64, int32_t f) {
        if (!(t64 >= 0.0 && t64 <= 1.0)) return;
        const float t = (float)t64;
        if (t < best_t[i] || (t == best_t[i] && f < best_f[i])) {
            best_t[i] = t;
            best_f[i] = f;
        }
    };

    // FP64 decision for one (face, direction pair) that passed the FP32 filter:
    // the segment-triangle test in the same expression order as the definition
    // (Moller-Trumbore), so both directions of the pair come out exactly as
    // separate evaluations would (negating D negates P, det and t exactly).
    auto decide64_tri = [&](int p, int j, double &tout) -> bool {
        const double a0 = s_f[0][j], a1 = s_f[1][j], a2 = s_f[2][j];
        const double E1[3] = {(double)s_f[3][j] - a0, (double)s_f[4][j] - a1, (double)s_f[5][j] - a2};
        const double E2[3] = {(double)s_f[6][j] - a0, (double)s_f[7][j] - a1, (double)s_f[8][j] - a2};
        const double T[3] = {(double)o[0] - a0, (double)o[1] - a1, (double)o[2] - a2};
        const double Dv[3] = {(double)s_dir[p][0], (double)s_dir[p][1], (double)s_dir[p][2]};
        const double P[3] = {Dv[1] * E2[2] - Dv[2] * E2[1], Dv[2] * E2[0] - Dv[0] * E2[2], Dv[0] * E2[1] - Dv[1] * E2[0]};
        const double det = E1[0] * P[0] + E1[1] * P[1] + E1[2] * P[2];
        if (det == 0.0) return false;
        const double u = (T[0] * P[0] + T[1] * P[1] + T[2] * P[2]) / det;
        if (u < 0.0 || u > 1.0) return false;
        const double Qv[3] = {T[1] * E1[2] - T[2] * E1[1], T[2] * E1[0] - T[0] * E1[2], T[0] * E1[1] - T[1] * E1[0]};
        const double v = (Dv[0] * Qv[0] + Dv[1] * Qv[1] + Dv[2] * Qv[2]) / det;
        if (v < 0.0 || u + v > 1.0) return false;
        tout = (E2[0] * Qv[0] + E2[1] * Qv[1] + E2[2] * Qv[2]) / det;
        return true;
    };
    auto decide64_seg = [&](int p, int j, double &tout) -> bool {
        const double a0 = s_f[0][j], a1 = s_f[1][j];
        const double e0 = (double)s_f[2][j] - a0, e1 = (double)s_f[3][j] - a1;
        const double D0 = (double)s_dir[p][0], D1 = (double)s_dir[p][1];
        const double den = D0 * e1 - D1 * e0;
        if (den == 0.0) return false;
        const double w0 = a0 - (double)o[0], w1 = a1 - (double)o[1];
        tout = (w0 * e1 - w1 * e0) / den;
        const double sp = (w0 * D1 - w1 * D0) / den;
        return sp >= 0.0 && sp <= 1.0;
    };
    // Runtime pair index p: one copy of the FP64 code; the result reaches the
    // register-resident best arrays through an unrolled predicated update.
    auto decide_mask = [&](uint32_t cm, int j, int32_t f) {
        while (cm) {
            const int p = __builtin_ctz(cm);
            cm &= cm - 1u;
            double t;
            bool hit;
            if constexpr (D == 3) hit = decide64_tri(p, j, t);
            else hit = decide64_seg(p, j, t);
            if (!hit) continue;
#pragma unroll
            for (int q = 0; q < NP; ++q)
                if (q == p) {
                    consider(2 * q, t, f);       // direction 1 + 2q
                    consider(2 * q + 1, -t, f);  // its opposite
                }
        }
    };

    // Staged faces are visited in batches of 64: each lane first marks the faces
    // whose box meets its link box (broadcast LDS reads), then walks only its
    // own marked faces, so lanes stay busy whatever the spatial mix.
    auto test_staged = [&](int n) {
        __syncthreads();
        if (valid)
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int jn = min(64, n - j0);
            uint64_t nm = 0;
            for (int jj = 0; jj < jn; ++jj) {
                bool near = true;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    const float mn = s_f[NF - 2 * D + a][j0 + jj], mx = s_f[NF - D + a][j0 + jj];
                    near = near && mn <= chi[a] && mx >= clo[a];
                }
                nm |= near ? (1ull << jj) : 0ull;
            }
            while (nm) {
                const int j = j0 + __builtin_ctzll(nm);
                nm &= nm - 1ull;
                const int32_t f = s_id[j];
                if constexpr (D == 3) {
                    // FP32 filter.  Each quantity below carries an absolute rounding error
                    // bounded by 2^-21 times the product of the L1 norms of its factors;
                    // margins of 2^-20 times those products keep every true hit.
                    const float T0 = o[0] - s_f[0][j], T1 = o[1] - s_f[1][j], T2 = o[2] - s_f[2][j];
                    const float e10 = s_f[3][j] - s_f[0][j], e11 = s_f[4][j] - s_f[1][j], e12 = s_f[5][j] - s_f[2][j];
                    const float e20 = s_f[6][j] - s_f[0][j], e21 = s_f[7][j] - s_f[1][j], e22 = s_f[8][j] - s_f[2][j];
                    const float n0 = s_f[9][j], n1 = s_f[10][j], n2 = s_f[11][j];
                    const float nT = fabsf(T0) + fabsf(T1) + fabsf(T2);
                    const float n1n = fabsf(e10) + fabsf(e11) + fabsf(e12);
                    const float n2n = fabsf(e20) + fabsf(e21) + fabsf(e22);
                    const float mx_ = fmaxf(fmaxf(A.dx[0], A.dx[1]), A.dx[2]) * 9.5367431640625e-07f;  // dx * 2^-20
                    const float MU = mx_ * nT * n2n;
                    const float MV = mx_ * n1n * nT;
                    const float MD = mx_ * n1n * n2n;
                    const float MT = 9.5367431640625e-07f * nT * n1n * n2n;
                    const float p10 = (T1 * e22 - T2 * e21) * A.dx[0];
                    const float p11 = (T2 * e20 - T0 * e22) * A.dx[1];
                    const float p12 = (T0 * e21 - T1 * e20) * A.dx[2];
                    const float p20 = (e11 * T2 - e12 * T1) * A.dx[0];
                    const float p21 = (e12 * T0 - e10 * T2) * A.dx[1];
                    const float p22 = (e10 * T1 - e11 * T0) * A.dx[2];
                    const float d0 = n0 * A.dx[0], d1 = n1 * A.dx[1], d2 = n2 * A.dx[2];
                    const float tn = (T0 * n0 + T1 * n1) + T2 * n2;
                    uint32_t cm = 0;   // direction pairs that pass the FP32 filter
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const int i = 1 + 2 * p;
                        const int c0 = dir_c<D>(i, 0), c1 = dir_c<D>(i, 1), c2 = dir_c<D>(i, 2);
                        float den = 0.0f, nu = 0.0f, nv = 0.0f;
                        if (c0) { den += c0 > 0 ? d0 : -d0; nu += c0 > 0 ? p10 : -p10; nv += c0 > 0 ? p20 : -p20; }
                        if (c1) { den += c1 > 0 ? d1 : -d1; nu += c1 > 0 ? p11 : -p11; nv += c1 > 0 ? p21 : -p21; }
                        if (c2) { den += c2 > 0 ? d2 : -d2; nu += c2 > 0 ? p12 : -p12; nv += c2 > 0 ? p22 : -p22; }
                        bool cand;
                        if (fabsf(den) <= MD) {
                            cand = true;   // grazing: the sign of the denominator is not known in FP32
                        } else {
                            const float ad = fabsf(den);
                            const float su = den < 0.0f ? -nu : nu;
                            const float sv = den < 0.0f ? -nv : nv;
                            const float st = den < 0.0f ? tn : -tn;   // sign(den) * (-tn) = t * |den|
                            const float lim = ad + MD + MT;
                            cand = su >= -MU && sv >= -MV && su + sv <= ad + MU + MV + MD &&
                                   ((st >= -MT && st <= lim) || (-st >= -MT && -st <= lim));
                        }
                        cm |= cand ? (1u << p) : 0u;
                    }
                    if (cm) decide_mask(cm, j, f);
                } else {
                    const float w0 = s_f[0][j] - o[0], w1 = s_f[1][j] - o[1];
                    const float e0 = s_f[2][j] - s_f[0][j], e1 = s_f[3][j] - s_f[1][j];
                    const float nw = fabsf(w0) + fabsf(w1), ne = fabsf(e0) + fabsf(e1);
                    const float mx_ = fmaxf(A.dx[0], A.dx[1]) * 9.5367431640625e-07f;
                    const float MD = mx_ * ne, MS = mx_ * nw, MW = 9.5367431640625e-07f * nw * ne;
                    const float wxe = w0 * e1 - w1 * e0;
                    uint32_t cm = 0;
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const int i = 1 + 2 * p;
                        const float D0 = (float)dir_c<D>(i, 0) * A.dx[0], D1 = (float)dir_c<D>(i, 1) * A.dx[1];
                        const float den = D0 * e1 - D1 * e0;
                        bool cand;
                        if (fabsf(den) <= MD) {
                            cand = true;
                        } else {
                            const float ad = fabsf(den);
                            const float sn = w0 * D1 - w1 * D0;
                            const float ss = den < 0.0f ? -sn : sn;
                            const float st = den < 0.0f ? -wxe : wxe;
                            const float lim = ad + MD + MW;
                            cand = ss >= -MS && ss <= ad + MS + MD &&
                                   ((st >= -MW && st <= lim) || (-st >= -MW && -st <= lim));
                        }
                        cm |= cand ? (1u << p) : 0u;
                    }
                    if (cm) decide_mask(cm, j, f);
                }
            }
        }
        __syncthreads();
    };

    int count = 0;
    for (int sb = 0; sb < BPW; ++sb) {
        if (first + sb >= A.n) break;
        int sc[3];
        sc[0] = __shfl(bc[0], sb * CELLS, 64);
        sc[1] = __shfl(bc[1], sb * CELLS, 64);
        sc[2] = __shfl(bc[2], sb * CELLS, 64);
        float qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
        int ilo[3] = {0, 0, 0}, ihi[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < D; ++a) {
            qlo[a] = (dev::cell_centre(A.lo[a], 4 * sc[a], A.dx[a]) - A.dx[a]) - A.eps[a];
            qhi[a] = (dev::cell_centre(A.lo[a], 4 * sc[a] + 3, A.dx[a]) + A.dx[a]) + A.eps[a];
            ilo[a] = dev::bin_of(qlo[a], A.bins.lo[a], A.bins.s[a], A.bins.B);
            ihi[a] = dev::bin_of(qhi[a], A.bins.lo[a], A.bins.s[a], A.bins.B);
        }
        for (int z = ilo[2]; z <= ihi[2]; ++z)
            for (int y = ilo[1]; y <= ihi[1]; ++y)
                for (int x = ilo[0]; x <= ihi[0]; ++x) {
                    const int64_t b = ((int64_t)z * A.bins.B + y) * A.bins.B + x;
                    const uint32_t s0 = A.bins.off[b], s1 = A.bins.off[b + 1];
                    for (uint32_t base = s0; base < s1; base += 64) {
                        const uint32_t j = base + lane;
                        bool keep = false;
                        int32_t f = -1;
                        float bb[6] = {0, 0, 0, 0, 0, 0};
                        if (j < s1) {
                            f = A.bins.ids[j];
                            keep = true;
                            const int cur[3] = {x, y, z};
#pragma unroll
                            for (int a = 0; a < D; ++a) {
                                bb[a] = A.faces.aabb[(int64_t)a * F + f];
                                bb[D + a] = A.faces.aabb[(int64_t)(D + a) * F + f];
                                const int fb = max(dev::bin_of(bb[a], A.bins.lo[a], A.bins.s[a], A.bins.B), ilo[a]);
                                keep = keep && fb == cur[a] && bb[a] <= qhi[a] && bb[D + a] >= qlo[a];
                            }
                        }
                        const uint64_t mask = __ballot(keep);
                        const int nk = __popcll(mask);
                        if (nk == 0) continue;
                        if (count + nk > kLinkCap) {
                            test_staged(count);
                            count = 0;
                        }
                        if (keep) {
                            const int pos = count + dev::lanes_below(mask);
                            s_id[pos] = f;
                            if constexpr (D == 3) {
                                float v[9];
#pragma unroll
                                for (int k = 0; k < 9; ++k) v[k] = A.faces.coords[(int64_t)k * F + f];
                                const float e10 = v[3] - v[0], e11 = v[4] - v[1], e12 = v[5] - v[2];
                                const float e20 = v[6] - v[0], e21 = v[7] - v[1], e22 = v[8] - v[2];
#pragma unroll
                                for (int k = 0; k < 9; ++k) s_f[k][pos] = v[k];
                                s_f[9][pos] = e11 * e22 - e12 * e21;
                                s_f[10][pos] = e12 * e20 - e10 * e22;
                                s_f[11][pos] = e10 * e21 - e11 * e20;
                            } else {
#pragma unroll
                                for (int k = 0; k < 4; ++k) s_f[k][pos] = A.faces.coords[(int64_t)k * F + f];
                            }
#pragma unroll
                            for (int a = 0; a < 2 * D; ++a) s_f[NF - 2 * D + a][pos] = bb[a];
                        }
                        count += nk;
                    }
                }
    }
    if (count > 0) test_staged(count);

    // ordered compaction of the cells that have a link
    bool has = false;
#pragma unroll
    for (int i = 0; i < Q - 1; ++i) has = has || best_f[i] >= 0;
    has = has && valid;
    const uint64_t hm = __ballot(has);
    // rank inside the block: lanes of this block below this lane that have a link
    const int sub = lane / CELLS;
    uint64_t bm = hm;
    if constexpr (CELLS < 64) bm = (hm >> (sub * CELLS)) & ((1ull << CELLS) - 1);
    if (valid && cell == 0) A.count[blk] = (uint32_t)__popcll(bm);
    if (has) {
        const int64_t node = blk * CELLS + __popcll(bm & ((1ull << cell) - 1));
        A.node_key[node] = (uint64_t)key * CELLS + (uint64_t)cell;
        float *qr = A.q + node * Q;
        int32_t *fr = A.face + node * Q;
        qr[0] = -1.0f;
        fr[0] = -1;
#pragma unroll
        for (int i = 0; i < Q - 1; ++i) {
            qr[i + 1] = best_f[i] >= 0 ? best_t[i] : -1.0f;
            fr[i + 1] = best_f[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint: one thread per (node, direction) slot.
// ---------------------------------------------------------------------------
template <int D, int Q>
struct AdjArgs {
    const float *coords;
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

constexpr int kAdjThreads = 256;   // one node per thread
constexpr int kAdjHash = 512;      // per-workgroup face accumulators

// Gradient of one link's t with respect to the D vertices of its face,
// scaled by w: out[k][a] = w * lambda_k * n_a / (D . n).
template <int D>
__device__ __forceinline__ void link_grad(const float *coords, int64_t F, int32_t f, const float o[3],
                                          const float Dv[3], float w, float out[D][D]) {
    if constexpr (D == 3) {
        float v[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] = coords[(int64_t)k * F + f];
        const float e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
        const float e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
        const float T[3] = {o[0] - v[0], o[1] - v[1], o[2] - v[2]};
        const float n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                            e1[0] * e2[1] - e1[1] * e2[0]};
        const float den = (Dv[0] * n[0] + Dv[1] * n[1]) + Dv[2] * n[2];
        const float dd = sqrtf((Dv[0] * Dv[0] + Dv[1] * Dv[1]) + Dv[2] * Dv[2]);
        const float ee = sqrtf((e1[0] * e1[0] + e1[1] * e1[1]) + e1[2] * e1[2]) *
                         sqrtf((e2[0] * e2[0] + e2[1] * e2[1]) + e2[2] * e2[2]);
        float u, vv, inv;
        if (fabsf(den) < 0.0009765625f * dd * ee) {
            // grazing ray: barycentrics and denominator in FP64 from the FP32 data
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
            const float p1[3] = {T[1] * e2[2] - T[2] * e2[1], T[2] * e2[0] - T[0] * e2[2],
                                 T[0] * e2[1] - T[1] * e2[0]};
            const float p2[3] = {e1[1] * T[2] - e1[2] * T[1], e1[2] * T[0] - e1[0] * T[2],
                                 e1[0] * T[1] - e1[1] * T[0]};
            inv = 1.0f / den;
            u = ((Dv[0] * p1[0] + Dv[1] * p1[1]) + Dv[2] * p1[2]) * inv;
            vv = ((Dv[0] * p2[0] + Dv[1] * p2[1]) + Dv[2] * p2[2]) * inv;
        }
        const float lam[3] = {1.0f - u - vv, u, vv};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float sc = w * lam[k] * inv;
#pragma unroll
            for (int a = 0; a < 3; ++a) out[k][a] = sc * n[a];
        }
    } else {
        const float a0 = coords[(int64_t)0 * F + f], a1 = coords[(int64_t)1 * F + f];
        const float b0 = coords[(int64_t)2 * F + f], b1 = coords[(int64_t)3 * F + f];
        const float e0 = b0 - a0, e1 = b1 - a1;
        const float n[2] = {-e1, e0};
        const float w0 = a0 - o[0], w1 = a1 - o[1];
        const float den = Dv[0] * n[0] + Dv[1] * n[1];
        const float dd = sqrtf(Dv[0] * Dv[0] + Dv[1] * Dv[1]);
        const float ee = sqrtf(e0 * e0 + e1 * e1);
        float sp, inv;
        if (fabsf(den) < 0.0009765625f * dd * ee) {
            const double E0 = (double)b0 - (double)a0, E1 = (double)b1 - (double)a1;
            const double W0 = (double)a0 - (double)o[0], W1 = (double)a1 - (double)o[1];
            const double dxe = (double)Dv[0] * E1 - (double)Dv[1] * E0;   // D x e
            sp = (float)((W0 * (double)Dv[1] - W1 * (double)Dv[0]) / dxe);
            inv = (float)(1.0 / ((double)Dv[0] * -E1 + (double)Dv[1] * E0));
        } else {
            const float dxe = Dv[0] * e1 - Dv[1] * e0;
            sp = (w0 * Dv[1] - w1 * Dv[0]) / dxe;
            inv = 1.0f / den;
        }
        const float lam[2] = {1.0f - sp, sp};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float sc = w * lam[k] * inv;
            out[k][0] = sc * n[0];
            out[k][1] = sc * n[1];
        }
    }
}

// One thread per node.  Contributions are summed per face in an LDS hash
// table first (neighbouring nodes in key order hit few distinct faces), then
// each face's sums go to its vertices with one float atomic per coordinate.
template <int D, int Q>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint(AdjArgs<D, Q> A) {
    constexpr int CELLS = D == 3 ? 64 : 16;
    __shared__ int32_t s_key[kAdjHash];
    __shared__ float s_acc[kAdjHash][D * D];
    for (int i = threadIdx.x; i < kAdjHash; i += kAdjThreads) {
        s_key[i] = -1;
#pragma unroll
        for (int c = 0; c < D * D; ++c) s_acc[i][c] = 0.0f;
    }
    __syncthreads();
    const int64_t node = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
    if (node < A.n) {
        const uint64_t nk = A.node_key[node];
        const uint32_t key = (uint32_t)(nk / CELLS);
        const int cell = (int)(nk % CELLS);
        int bc[3];
        dev::decode_key<D>(key, A.level, A.R[0], A.R[1], bc);
        float o[3];
        o[0] = dev::cell_centre(A.lo[0], 4 * bc[0] + (cell & 3), A.dx[0]);
        o[1] = dev::cell_centre(A.lo[1], 4 * bc[1] + ((cell >> 2) & 3), A.dx[1]);
        o[2] = D == 3 ? dev::cell_centre(A.lo[2], 4 * bc[2] + (cell >> 4), A.dx[2]) : 0.0f;
        for (int i = 1; i < Q; ++i) {
            const int32_t f = A.face[node * Q + i];
            const float w = A.gq[node * Q + i];
            if (f < 0 || w == 0.0f) continue;
            float Dv[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) Dv[a] = (float)(D == 3 ? kDir3[i][a] : kDir2[i][a]) * A.dx[a];
            float g[D][D];
            link_grad<D>(A.coords, A.F, f, o, Dv, w, g);
            uint32_t h = ((uint32_t)f * 2654435761u) >> 23;   // 9 bits: kAdjHash slots
            int slot = -1;
            for (int probe = 0; probe < kAdjHash; ++probe) {
                const int32_t prev = atomicCAS(&s_key[h], -1, f);
                if (prev == -1 || prev == f) {
                    slot = (int)h;
                    break;
                }
                h = (h + 1) & (kAdjHash - 1);
            }
            if (slot >= 0) {
#pragma unroll
                for (int k = 0; k < D; ++k)
#pragma unroll
                    for (int a = 0; a < D; ++a) atomicAdd(&s_acc[slot][k * D + a], g[k][a]);
            } else {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const int64_t vk = A.fidx[(int64_t)f * D + k];
#pragma unroll
                    for (int a = 0; a < D; ++a) unsafeAtomicAdd(&A.grad[vk * D + a], g[k][a]);
                }
            }
        }
    }
    __syncthreads();
    for (int sl = threadIdx.x; sl < kAdjHash; sl += kAdjThreads) {
        const int32_t f = s_key[sl];
        if (f < 0) continue;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int64_t vk = A.fidx[(int64_t)f * D + k];
#pragma unroll
            for (int a = 0; a < D; ++a) unsafeAtomicAdd(&A.grad[vk * D + a], s_acc[sl][k * D + a]);
        }
    }
}

// Staged nodes of block b (rows b*4^D .. b*4^D + count[b]) -> rows off[b].. of
// the output; one wave per block, rows copied as flat coalesced runs.
template <int Q, int CELLS>
__global__ __launch_bounds__(64) void k_compact_nodes(const uint32_t *count, const uint32_t *off, int64_t nblk,
                                                      const uint64_t *skey, const float *sq, const int32_t *sface,
                                                      uint64_t *key, float *q, int32_t *face) {
    const int64_t b = blockIdx.x;
    if (b >= nblk) return;
    const int c = (int)count[b];
    if (c == 0) return;
    const int64_t src = b * CELLS, dst = off[b];
    for (int r = threadIdx.x; r < c; r += 64) key[dst + r] = skey[src + r];
    for (int e = threadIdx.x; e < c * Q; e += 64) {
        q[dst * Q + e] = sq[src * Q + e];
        face[dst * Q + e] = sface[src * Q + e];
    }
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
        uint64_t *key = nullptr;
        float *q = nullptr;
        int32_t *face = nullptr;
        ~Staging() {
            dev_free(ctx->mem, count, s);
            dev_free(ctx->mem, off, s);
            dev_free(ctx->mem, key, s);
            dev_free(ctx->mem, q, s);
            dev_free(ctx->mem, face, s);
        }
    } st{ctx, s};
    AGAL_TRY(dev_alloc(ctx->mem, &st.count, (size_t)LL.n, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.off, (size_t)LL.n + 1, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.key, (size_t)cap, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.q, (size_t)cap * Q, s));
    AGAL_TRY(dev_alloc(ctx->mem, &st.face, (size_t)cap * Q, s));
    LinkArgs<D, Q> A{};
    A.faces = dev::Faces{g->coords, g->aabb, g->F};
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
    A.count = st.count;
    A.node_key = st.key;
    A.q = st.q;
    A.face = st.face;
    const int64_t waves = (LL.n + BPW - 1) / BPW;
    {
        ProfScope prof(ctx, "q_links", s);
        hipLaunchKernelGGL((k_links<D, Q>), dim3((unsigned)waves), dim3(64), 0, s, A);
    }
    AGAL_TRY_HIP(hipGetLastError());
    AGAL_TRY(scan_u32(ctx, st.count, st.off, LL.n, s));
    uint32_t nn = 0;
    const uint32_t *src[1] = {st.off + LL.n};
    AGAL_TRY(read_back_u32(ctx, src, 1, &nn, s));
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
    A.coords = g->coords;
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
