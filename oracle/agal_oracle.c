/*
 * agal_oracle.c -- plain, serial, slow CPU oracle for the near-wall
 * mesh-adaptation path of "Towards a GPU-native adaptive mesh refinement
 * scheme for the Lattice Boltzmann Method in complex geometries"
 * (Jaber, Essel, Sullivan, 2025).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared.
 * On x86-64 every float expression below is evaluated in IEEE single
 * precision (SSE, FLT_EVAL_METHOD == 0) with no contraction into FMA, so the
 * FP32 parts (bins, cell centres, the separating-axis predicate) are a fixed
 * sequence of correctly rounded operations.  Link fractions, the adjoint and
 * the finite-difference harness run in FP64 on the FP32 inputs promoted
 * exactly.
 *
 * What each part follows:
 *  - import (index lists -> coordinate list): paper, Sec. II-B and the
 *    index/coordinate-list figure.
 *  - binning: paper, Sec. II-C-3 (bins of user density B over the initial
 *    grid, three arrays: ids grouped by bin, per-bin counts, first index).
 *    Bin membership here is the face's axis-aligned bounding box (every bin
 *    the box touches), ids ascending inside a bin.
 *  - flagging: paper, Sec. II-C-1/II-C-2: every cell of every block of a
 *    level tests adjacency to the faces of its bins; a block is marked when
 *    one of its cells is adjacent.  Adjacency is the closed-box reading: the
 *    face meets the closed cube of half-width d centred on the cell centre,
 *    decided by the 13-axis separating-axis test (the L-infinity form of the
 *    paper's distance criterion).
 *  - own-bin flagging (orc_refine_own_bin): the paper's own form, Sec.
 *    II-C-2 with Algorithm 1 and the propagation paragraph of Sec. II-C-3: a
 *    cell is flagged when its centre lies within Euclidean distance d of a
 *    face of the one bin holding the centre, then the marks spread over
 *    1 + floor(d / block length) rings of neighbouring blocks.
 *  - refinement: Sec. II-A (forest of octrees, blocks of 4^D cells, one level
 *    at a time) and Sec. II-C-1 (marked blocks are subdivided); 2:1 balance
 *    across faces, edges and corners is closed by a downward ripple.
 *  - link fractions: Sec. II-C-1 (cells find links with faces along each
 *    lattice direction): q is the fraction of the segment x -> x + c_i dx at
 *    which it first meets a face (closed faces, two-sided).
 *  - adjoint: derivative of q with respect to the vertices of the hit face,
 *    dq/dv_k = lambda_k n / (Dv . n).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXL 8

static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory (%zu bytes)\n", n); abort(); }
    return p;
}
static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s ? s : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}
static void *xrealloc(void *p, size_t n) {
    void *q = realloc(p, n ? n : 1);
    if (!q) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return q;
}

static float fmin2(float a, float b) { return a < b ? a : b; }
static float fmax2(float a, float b) { return a > b ? a : b; }
static float fabs1(float a) { return a < 0.0f ? -a : a; }

/* ------------------------------------------------------------------ */
/* Lattice velocity sets.  Order: rest; axis directions in +/- pairs;   */
/* then (3D) the 12 edge directions in +/- pairs; then (D3Q27) the 8    */
/* corner directions in +/- pairs.  D2Q9: rest, (+-1,0), (0,+-1), then  */
/* the diagonals in +/- pairs.                                          */
/* ------------------------------------------------------------------ */
static const int D2Q9_C[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const int D3Q27_C[27][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

/* Fills c[Q][3]; returns the lattice's dimension or -1. */
int orc_lattice(int Q, int *c) {
    const int (*src)[3];
    int dim;
    if (Q == 9) { src = D2Q9_C; dim = 2; }
    else if (Q == 19 || Q == 27) { src = D3Q27_C; dim = 3; }
    else return -1;
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < 3; ++a) c[3 * i + a] = src[i][a];
    return dim;
}

/* ------------------------------------------------------------------ */
/* Import: index lists -> coordinate list                               */
/* coords[(f*dim + k)*dim + a] = verts[faces[f*dim+k]*dim + a]          */
/* ------------------------------------------------------------------ */
void orc_gather(int dim, const float *verts, const int32_t *faces, int64_t F, float *coords) {
    for (int64_t f = 0; f < F; ++f)
        for (int k = 0; k < dim; ++k)
            for (int a = 0; a < dim; ++a)
                coords[(f * dim + k) * dim + a] = verts[(int64_t)faces[f * dim + k] * dim + a];
}

/* ------------------------------------------------------------------ */
/* Bins (FP32)                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    int dim, B;
    float lo[3], hi[3], s[3];
    int64_t nb, P;
    uint32_t *count, *off;
    int32_t *ids;
} orc_bins;

/* Bin index of coordinate x along one axis: floor((x - lo) * s), clamped to [0, B-1]
 * (clamped in float before the integer conversion so any finite x is defined). */
static int bin_index(float x, float lo, float s, int B) {
    float t = (x - lo) * s;
    float f = floorf(t);
    if (f < 0.0f) return 0;
    if (f > (float)(B - 1)) return B - 1;
    return (int)f;
}

static void face_bin_range(const orc_bins *bn, const float *fc, int lo_i[3], int hi_i[3]) {
    int dim = bn->dim;
    for (int a = 0; a < 3; ++a) { lo_i[a] = 0; hi_i[a] = 0; }
    for (int a = 0; a < dim; ++a) {
        float mn = fc[a], mx = fc[a];
        for (int k = 1; k < dim; ++k) {
            mn = fmin2(mn, fc[k * dim + a]);
            mx = fmax2(mx, fc[k * dim + a]);
        }
        lo_i[a] = bin_index(mn, bn->lo[a], bn->s[a], bn->B);
        hi_i[a] = bin_index(mx, bn->lo[a], bn->s[a], bn->B);
    }
}

orc_bins *orc_bin_faces(int dim, const float *coords, int64_t F, const float *lo, const float *hi, int B) {
    if (B < 1 || (dim != 2 && dim != 3)) return NULL;
    orc_bins *bn = (orc_bins *)xcalloc(1, sizeof(orc_bins));
    bn->dim = dim;
    bn->B = B;
    bn->nb = 1;
    for (int a = 0; a < 3; ++a) {
        bn->lo[a] = a < dim ? lo[a] : 0.0f;
        bn->hi[a] = a < dim ? hi[a] : 1.0f;
        bn->s[a] = (float)B / (bn->hi[a] - bn->lo[a]);
        if (a < dim) bn->nb *= B;
    }
    bn->count = (uint32_t *)xcalloc((size_t)bn->nb, sizeof(uint32_t));
    bn->off = (uint32_t *)xcalloc((size_t)bn->nb + 1, sizeof(uint32_t));
    /* pass 1: count */
    for (int64_t f = 0; f < F; ++f) {
        int l[3], h[3];
        face_bin_range(bn, coords + f * dim * dim, l, h);
        for (int z = l[2]; z <= h[2]; ++z)
            for (int y = l[1]; y <= h[1]; ++y)
                for (int x = l[0]; x <= h[0]; ++x)
                    bn->count[((int64_t)z * B + y) * B + x] += 1;
    }
    /* exclusive scan */
    uint64_t run = 0;
    for (int64_t b = 0; b < bn->nb; ++b) { bn->off[b] = (uint32_t)run; run += bn->count[b]; }
    bn->off[bn->nb] = (uint32_t)run;
    bn->P = (int64_t)run;
    /* pass 2: append in ascending face order */
    bn->ids = (int32_t *)xmalloc((size_t)bn->P * sizeof(int32_t));
    uint32_t *cur = (uint32_t *)xcalloc((size_t)bn->nb, sizeof(uint32_t));
    for (int64_t f = 0; f < F; ++f) {
        int l[3], h[3];
        face_bin_range(bn, coords + f * dim * dim, l, h);
        for (int z = l[2]; z <= h[2]; ++z)
            for (int y = l[1]; y <= h[1]; ++y)
                for (int x = l[0]; x <= h[0]; ++x) {
                    int64_t b = ((int64_t)z * B + y) * B + x;
                    bn->ids[bn->off[b] + cur[b]++] = (int32_t)f;
                }
    }
    free(cur);
    return bn;
}

/*
 * The paper's own binning (Sec. II-C-3, spatial binning and its
 * discretization figure): every face is sampled at points whose number grows
 * with its size, and it is assigned to each bin holding at least one point.
 * An edge from a to b, e = b - a, is cut into 2^k equal pieces, k the least
 * integer >= 0 with max_a |e_a| <= spacing * 2^k (k at most ORC_DISC_KMAX); its
 * points are a + e * (j * 2^-k), j = 0 .. 2^k, each component one FP32
 * product and one FP32 sum.  A triangle (a, b, c) takes the points q_j of its
 * edge a -> b, and every segment q_j -> c is sampled the same way (its own k).
 * A 2D face is its edge.  Points go to bins by the same index function as the
 * box binning.  Output layout as orc_bin_faces: per bin, ascending face ids.
 */
#define ORC_DISC_KMAX 12

static int disc_k(const float *e, int dim, float spacing) {
    float s = 0.0f;
    for (int a = 0; a < dim; ++a) s = fmax2(s, fabsf(e[a]));
    int k = 0;
    while (k < ORC_DISC_KMAX && !(s <= ldexpf(spacing, k))) ++k;
    return k;
}

/* visits every sample point of face fc, calling add(bin) */
static void disc_visit(const orc_bins *bn, const float *fc, float spacing, int64_t *list, int64_t *nlist,
                       int64_t *stamp, int64_t mark) {
    int dim = bn->dim, B = bn->B;
    const float *a = fc, *b = fc + dim;
    float e[3] = {0, 0, 0};
    for (int x = 0; x < dim; ++x) e[x] = b[x] - a[x];
    int k1 = disc_k(e, dim, spacing);
    int64_t n1 = (int64_t)1 << k1;
    for (int64_t j = 0; j <= n1; ++j) {
        float t = ldexpf((float)j, -k1);
        float q[3] = {0, 0, 0};
        for (int x = 0; x < dim; ++x) q[x] = a[x] + e[x] * t;
        float g[3] = {0, 0, 0};
        int k2 = 0;
        if (dim == 3) {
            for (int x = 0; x < 3; ++x) g[x] = fc[6 + x] - q[x];
            k2 = disc_k(g, 3, spacing);
        }
        int64_t n2 = dim == 3 ? ((int64_t)1 << k2) : 0;
        for (int64_t i = 0; i <= n2; ++i) {
            float p[3] = {0, 0, 0};
            if (dim == 3) {
                float u = ldexpf((float)i, -k2);
                for (int x = 0; x < 3; ++x) p[x] = q[x] + g[x] * u;
            } else {
                p[0] = q[0];
                p[1] = q[1];
            }
            int ix[3] = {0, 0, 0};
            for (int x = 0; x < dim; ++x) ix[x] = bin_index(p[x], bn->lo[x], bn->s[x], B);
            int64_t bb = ((int64_t)ix[2] * B + ix[1]) * B + ix[0];
            if (stamp[bb] != mark) {
                stamp[bb] = mark;
                list[(*nlist)++] = bb;
            }
        }
    }
}

static int cmp_i64(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

orc_bins *orc_bin_faces_discrete(int dim, const float *coords, int64_t F, const float *lo, const float *hi, int B,
                                 float spacing) {
    if (B < 1 || (dim != 2 && dim != 3) || !(spacing > 0.0f)) return NULL;
    orc_bins *bn = (orc_bins *)xcalloc(1, sizeof(orc_bins));
    bn->dim = dim;
    bn->B = B;
    bn->nb = 1;
    for (int a = 0; a < 3; ++a) {
        bn->lo[a] = a < dim ? lo[a] : 0.0f;
        bn->hi[a] = a < dim ? hi[a] : 1.0f;
        bn->s[a] = (float)B / (bn->hi[a] - bn->lo[a]);
        if (a < dim) bn->nb *= B;
    }
    bn->count = (uint32_t *)xcalloc((size_t)bn->nb, sizeof(uint32_t));
    bn->off = (uint32_t *)xcalloc((size_t)bn->nb + 1, sizeof(uint32_t));
    int64_t *stamp = (int64_t *)xmalloc((size_t)bn->nb * sizeof(int64_t));
    for (int64_t b = 0; b < bn->nb; ++b) stamp[b] = -1;
    /* the distinct bins of each face, face by face */
    int64_t cap = 1024, n = 0;
    int64_t *pairs_bin = (int64_t *)xmalloc((size_t)cap * sizeof(int64_t));
    int64_t *pairs_face = (int64_t *)xmalloc((size_t)cap * sizeof(int64_t));
    int64_t *list = (int64_t *)xmalloc((size_t)bn->nb * sizeof(int64_t));
    for (int64_t f = 0; f < F; ++f) {
        int64_t nl = 0;
        disc_visit(bn, coords + f * dim * dim, spacing, list, &nl, stamp, f);
        qsort(list, (size_t)nl, sizeof(int64_t), cmp_i64);
        for (int64_t i = 0; i < nl; ++i) {
            if (n == cap) {
                cap *= 2;
                pairs_bin = (int64_t *)xrealloc(pairs_bin, (size_t)cap * sizeof(int64_t));
                pairs_face = (int64_t *)xrealloc(pairs_face, (size_t)cap * sizeof(int64_t));
            }
            pairs_bin[n] = list[i];
            pairs_face[n] = f;
            ++n;
            bn->count[list[i]] += 1;
        }
    }
    uint64_t run = 0;
    for (int64_t b = 0; b < bn->nb; ++b) { bn->off[b] = (uint32_t)run; run += bn->count[b]; }
    bn->off[bn->nb] = (uint32_t)run;
    bn->P = (int64_t)run;
    bn->ids = (int32_t *)xmalloc((size_t)(bn->P > 0 ? bn->P : 1) * sizeof(int32_t));
    uint32_t *cur = (uint32_t *)xcalloc((size_t)bn->nb, sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {   /* pairs are in ascending face order */
        int64_t b = pairs_bin[i];
        bn->ids[bn->off[b] + cur[b]++] = (int32_t)pairs_face[i];
    }
    free(cur); free(stamp); free(list); free(pairs_bin); free(pairs_face);
    return bn;
}

void orc_bins_free(orc_bins *bn) {
    if (!bn) return;
    free(bn->count); free(bn->off); free(bn->ids); free(bn);
}
int64_t orc_bins_nb(const orc_bins *bn) { return bn->nb; }
int64_t orc_bins_P(const orc_bins *bn) { return bn->P; }
const uint32_t *orc_bins_count(const orc_bins *bn) { return bn->count; }
const uint32_t *orc_bins_off(const orc_bins *bn) { return bn->off; }
const int32_t *orc_bins_ids(const orc_bins *bn) { return bn->ids; }

/* ------------------------------------------------------------------ */
/* Separating-axis predicate (FP32, closed sets).  Returns 1 when the  */
/* face meets the closed cube [m-h, m+h]^D, 0 when an axis separates    */
/* them (strict '>' only).                                              */
/* ------------------------------------------------------------------ */
static int sep_interval3(float p0, float p1, float p2, float r) {
    float mn = fmin2(fmin2(p0, p1), p2);
    float mx = fmax2(fmax2(p0, p1), p2);
    return (mn > r) || (mx < -r);
}

static int sat_tri(const float *v, const float *m, float h) {
    float A[3], Bv[3], C[3];
    for (int a = 0; a < 3; ++a) {
        A[a] = v[0 * 3 + a] - m[a];
        Bv[a] = v[1 * 3 + a] - m[a];
        C[a] = v[2 * 3 + a] - m[a];
    }
    /* the three box axes */
    for (int a = 0; a < 3; ++a)
        if (sep_interval3(A[a], Bv[a], C[a], h)) return 0;
    float E0[3], E1[3], E2[3];
    for (int a = 0; a < 3; ++a) {
        E0[a] = Bv[a] - A[a];
        E1[a] = C[a] - Bv[a];
        E2[a] = A[a] - C[a];
    }
    /* the face normal N = E0 x E1 */
    float N[3];
    N[0] = E0[1] * E1[2] - E0[2] * E1[1];
    N[1] = E0[2] * E1[0] - E0[0] * E1[2];
    N[2] = E0[0] * E1[1] - E0[1] * E1[0];
    float s = (N[0] * A[0] + N[1] * A[1]) + N[2] * A[2];
    float r = h * ((fabs1(N[0]) + fabs1(N[1])) + fabs1(N[2]));
    if (s > r || s < -r) return 0;
    /* nine edge-cross-axis axes: e_k x E for k in {x,y,z}, E in {E0,E1,E2} */
    const float *E[3] = {E0, E1, E2};
    const float *P[3] = {A, Bv, C};
    for (int j = 0; j < 3; ++j) {
        const float *e = E[j];
        for (int k = 0; k < 3; ++k) {
            /* nonzero components (u, v) of e_k x e, in increasing axis order */
            int iu, iv;
            float au, av;
            if (k == 0) { iu = 1; iv = 2; au = -e[2]; av = e[1]; }
            else if (k == 1) { iu = 0; iv = 2; au = e[2]; av = -e[0]; }
            else { iu = 0; iv = 1; au = -e[1]; av = e[0]; }
            float p0 = au * P[0][iu] + av * P[0][iv];
            float p1 = au * P[1][iu] + av * P[1][iv];
            float p2 = au * P[2][iu] + av * P[2][iv];
            float rr = h * (fabs1(au) + fabs1(av));
            if (sep_interval3(p0, p1, p2, rr)) return 0;
        }
    }
    return 1;
}

static int sat_seg(const float *v, const float *m, float h) {
    float A[2], Bv[2];
    for (int a = 0; a < 2; ++a) {
        A[a] = v[0 * 2 + a] - m[a];
        Bv[a] = v[1 * 2 + a] - m[a];
    }
    for (int a = 0; a < 2; ++a) {
        float mn = fmin2(A[a], Bv[a]), mx = fmax2(A[a], Bv[a]);
        if (mn > h || mx < -h) return 0;
    }
    float Nx = -(Bv[1] - A[1]);
    float Ny = Bv[0] - A[0];
    float pA = Nx * A[0] + Ny * A[1];
    float pB = Nx * Bv[0] + Ny * Bv[1];
    float r = h * (fabs1(Nx) + fabs1(Ny));
    float mn = fmin2(pA, pB), mx = fmax2(pA, pB);
    if (mn > r || mx < -r) return 0;
    return 1;
}

int orc_sat(int dim, const float *face, const float *m, float h) {
    return dim == 3 ? sat_tri(face, m, h) : sat_seg(face, m, h);
}

/* ------------------------------------------------------------------ */
/* Point within distance R of a face (Sec. II-C-2, Algorithm 1).  The   */
/* paper's region -- three vertex spheres, three edge cylinders and a   */
/* prism over the face (2D: two discs and a rectangle) -- is the set of */
/* points whose Euclidean distance to the closed face is at most R, so  */
/* it is decided here from that distance: the nearest point of a closed */
/* triangle lies on one of its three closed edges or, when the point    */
/* projects into the triangle, at that projection.                      */
/* ------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Squared distance from p to the closed segment [a, b] (dim 2 or 3), FP64. */
static double seg_dist2_d(int dim, const double *a, const double *b, const double *p) {
    double w[3] = {0, 0, 0}, e[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) { w[k] = p[k] - a[k]; e[k] = b[k] - a[k]; }
    double ee = dot3(e, e), we = dot3(w, e);
    double s = ee > 0.0 ? we / ee : 0.0;          /* parameter of the nearest point */
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    double r[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) r[k] = p[k] - (a[k] + s * e[k]);
    return dot3(r, r);
}

/* Squared Euclidean distance from p to the closed face v (2D segment or 3D
 * triangle), FP64. */
double orc_face_dist2(int dim, const double *v, const double *p) {
    if (dim == 2) return seg_dist2_d(2, v, v + 2, p);
    double best = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double d = seg_dist2_d(3, v + 3 * k, v + 3 * ((k + 1) % 3), p);
        if (d < best) best = d;
    }
    double e1[3], e2[3], n[3], w[3];
    for (int a = 0; a < 3; ++a) { e1[a] = v[3 + a] - v[a]; e2[a] = v[6 + a] - v[a]; w[a] = p[a] - v[a]; }
    cross3(e1, e2, n);
    double nn = dot3(n, n);
    if (nn > 0.0) {
        /* projection of p onto the plane, in the barycentric frame of (e1, e2) */
        double h = dot3(w, n) / nn;
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = w[a] - h * n[a];
        double c1[3], c2[3];
        cross3(x, e2, c1);
        cross3(e1, x, c2);
        double u = dot3(c1, n) / nn, t = dot3(c2, n) / nn;
        if (u >= 0.0 && t >= 0.0 && u + t <= 1.0) {
            double d = h * h * nn;
            if (d < best) best = d;
        }
    }
    return best;
}

int orc_near_face_l2(int dim, const double *v, const double *p, double R) {
    return orc_face_dist2(dim, v, p) <= R * R;
}

/* The same decision in FP32 as a fixed sequence of rounded operations (the
 * flag step of the own-bin refinement mode compares against it bit for bit).
 * No division: a squared distance d2 = c / m is compared as c <= R^2 m.
 *   R2 = R * R
 *   each closed edge [a, b] (2D: the segment; 3D: (v0,v1), (v1,v2), (v2,v0)):
 *     w = p - a, e = b - a, we = w.e
 *     we <= 0        -> near when w.w <= R2            (nearest point a)
 *     we >= e.e      -> near when u.u <= R2, u = p - b (nearest point b)
 *     otherwise      -> near when |e x w|^2 <= R2 (e.e)  (2D: (e0 w1 - e1 w0)^2)
 *   3D interior: n = (v1 - v0) x (v2 - v0), nn = n.n; when nn > 0 and
 *     ((v_{k+1} - v_k) x (p - v_k)) . n >= 0 for k = 0, 1, 2, near when
 *     ((p - v0) . n)^2 <= R2 nn.
 * Dot products are (x0 y0 + x1 y1) + x2 y2; cross products c0 = a1 b2 - a2 b1,
 * c1 = a2 b0 - a0 b2, c2 = a0 b1 - a1 b0. */
static float dot3f(const float *a, const float *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
static void cross3f(const float *a, const float *b, float *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static int edge_near_f(int dim, const float *a, const float *b, const float *p, float R2) {
    float w[3] = {0, 0, 0}, e[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) { w[k] = p[k] - a[k]; e[k] = b[k] - a[k]; }
    float we = dim == 3 ? dot3f(w, e) : w[0] * e[0] + w[1] * e[1];
    if (we <= 0.0f) {
        float ww = dim == 3 ? dot3f(w, w) : w[0] * w[0] + w[1] * w[1];
        return ww <= R2;
    }
    float ee = dim == 3 ? dot3f(e, e) : e[0] * e[0] + e[1] * e[1];
    if (we >= ee) {
        float u[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) u[k] = p[k] - b[k];
        float uu = dim == 3 ? dot3f(u, u) : u[0] * u[0] + u[1] * u[1];
        return uu <= R2;
    }
    float cc;
    if (dim == 3) {
        float c[3];
        cross3f(e, w, c);
        cc = dot3f(c, c);
    } else {
        float cr = e[0] * w[1] - e[1] * w[0];
        cc = cr * cr;
    }
    return cc <= R2 * ee;
}

int orc_near_l2_f32(int dim, const float *v, const float *p, float R) {
    float R2 = R * R;
    if (dim == 2) return edge_near_f(2, v, v + 2, p, R2);
    for (int k = 0; k < 3; ++k)
        if (edge_near_f(3, v + 3 * k, v + 3 * ((k + 1) % 3), p, R2)) return 1;
    float e1[3], e2[3], n[3];
    for (int a = 0; a < 3; ++a) { e1[a] = v[3 + a] - v[a]; e2[a] = v[6 + a] - v[a]; }
    cross3f(e1, e2, n);
    float nn = dot3f(n, n);
    if (!(nn > 0.0f)) return 0;
    for (int k = 0; k < 3; ++k) {
        float e[3], w[3], c[3];
        const float *a = v + 3 * k, *b = v + 3 * ((k + 1) % 3);
        for (int j = 0; j < 3; ++j) { e[j] = b[j] - a[j]; w[j] = p[j] - a[j]; }
        cross3f(e, w, c);
        if (!(dot3f(c, n) >= 0.0f)) return 0;
    }
    float w0[3];
    for (int j = 0; j < 3; ++j) w0[j] = p[j] - v[j];
    float hh = dot3f(w0, n);
    return hh * hh <= R2 * nn;
}

/* ------------------------------------------------------------------ */
/* Forest of quadtrees/octrees.  Roots form an R_x x R_y (x R_z) grid;  */
/* each tree node is a block of 4^D cells.  Block keys are hierarchical:*/
/* a root's key is its x-fastest linear index, a child's key is          */
/* parent_key * 2^D + child index (x-fastest), so sorting the keys of   */
/* one level orders its blocks root by root and Morton order inside.    */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t key;
    int32_t c[3];       /* block coordinates at its level */
    uint8_t leaf, mark, pass_mark;
    uint8_t cf[64];     /* per-cell flag (tested blocks only) */
} orc_block;

typedef struct { orc_block *b; int64_t n, cap; } orc_level;

typedef struct orc_forest {
    int dim, L;
    int roots[3];
    float lo[3], hi[3];
    float dx[ORC_MAXL + 1][3];
    float d[ORC_MAXL];
    orc_level lev[ORC_MAXL + 1];
    int64_t tests[ORC_MAXL + 1];
    /* exported arrays */
    uint32_t *ek[ORC_MAXL + 1];
    uint8_t *eleaf[ORC_MAXL + 1], *emark[ORC_MAXL + 1], *ecf[ORC_MAXL + 1];
} orc_forest;

static uint32_t key_of(const orc_forest *fo, int level, const int32_t *c) {
    uint32_t r0 = (uint32_t)(c[0] >> level), r1 = (uint32_t)(c[1] >> level), r2 = 0;
    if (fo->dim == 3) r2 = (uint32_t)(c[2] >> level);
    uint32_t key = (r2 * (uint32_t)fo->roots[1] + r1) * (uint32_t)fo->roots[0] + r0;
    for (int j = level - 1; j >= 0; --j) {
        uint32_t ci = (uint32_t)((c[0] >> j) & 1) | ((uint32_t)((c[1] >> j) & 1) << 1);
        if (fo->dim == 3) ci |= (uint32_t)((c[2] >> j) & 1) << 2;
        key = key * (fo->dim == 3 ? 8u : 4u) + ci;
    }
    return key;
}

static void level_push(orc_level *lv, const orc_block *b) {
    if (lv->n == lv->cap) {
        lv->cap = lv->cap ? 2 * lv->cap : 64;
        lv->b = (orc_block *)xrealloc(lv->b, (size_t)lv->cap * sizeof(orc_block));
    }
    lv->b[lv->n++] = *b;
}

static int cmp_block(const void *x, const void *y) {
    uint32_t a = ((const orc_block *)x)->key, b = ((const orc_block *)y)->key;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static orc_block *level_find(orc_level *lv, uint32_t key) {
    int64_t lo = 0, hi = lv->n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        uint32_t k = lv->b[mid].key;
        if (k == key) return &lv->b[mid];
        if (k < key) lo = mid + 1; else hi = mid - 1;
    }
    return NULL;
}

/* Cell centre: m_a = lo_a + (float)(2 g_a + 1) * (0.5f * dx_a) with g = 4*block + cell. */
static void cell_center(const orc_forest *fo, int level, const int32_t *bc, int cell, float *m) {
    int cc[3] = {cell & 3, (cell >> 2) & 3, (cell >> 4) & 3};
    for (int a = 0; a < fo->dim; ++a) {
        int32_t g = 4 * bc[a] + cc[a];
        m[a] = fo->lo[a] + (float)(2 * g + 1) * (0.5f * fo->dx[level][a]);
    }
}

static const float ORC_EPS = 9.5367431640625e-07f; /* 2^-20 */

/* Does any face of the candidate set meet the closed cube [m-h, m+h]? */
static int cell_flag(const orc_forest *fo, const float *coords, int64_t F, const orc_bins *bn,
                     const float *m, float h, int64_t *ntests) {
    int dim = fo->dim;
    if (!bn) {
        *ntests += F;
        for (int64_t f = 0; f < F; ++f)
            if (orc_sat(dim, coords + f * dim * dim, m, h)) return 1;
        return 0;
    }
    int l[3] = {0, 0, 0}, u[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        float qlo = (m[a] - h) - ORC_EPS;
        float qhi = (m[a] + h) + ORC_EPS;
        l[a] = bin_index(qlo, bn->lo[a], bn->s[a], bn->B);
        u[a] = bin_index(qhi, bn->lo[a], bn->s[a], bn->B);
    }
    int B = bn->B, hit = 0;
    for (int z = l[2]; z <= u[2]; ++z)
        for (int y = l[1]; y <= u[1]; ++y)
            for (int x = l[0]; x <= u[0]; ++x) {
                int64_t b = ((int64_t)z * B + y) * B + x;
                *ntests += bn->count[b];
                if (hit) continue;
                for (uint32_t j = bn->off[b]; j < bn->off[b + 1]; ++j) {
                    int32_t f = bn->ids[j];
                    if (orc_sat(dim, coords + (int64_t)f * dim * dim, m, h)) { hit = 1; break; }
                }
            }
    return hit;
}

/* Own-bin form of the flag (Sec. II-C-2, II-C-3): the cell looks only at the
 * faces of the one bin that holds its centre and is flagged when its centre
 * lies within distance R of one of them (FP32 decision above).  With B = 1
 * the bin holds every face (the paper's naive scheme). */
static int cell_flag_own_bin(const orc_forest *fo, const float *coords, const orc_bins *bn, const float *m, float R,
                             int64_t *ntests) {
    int dim = fo->dim;
    int ix[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) ix[a] = bin_index(m[a], bn->lo[a], bn->s[a], bn->B);
    int64_t b = ((int64_t)ix[2] * bn->B + ix[1]) * bn->B + ix[0];
    *ntests += bn->count[b];
    for (uint32_t j = bn->off[b]; j < bn->off[b + 1]; ++j)
        if (orc_near_l2_f32(dim, coords + (int64_t)bn->ids[j] * dim * dim, m, R)) return 1;
    return 0;
}

/* Number of propagation steps of a pass (Sec. II-C-3): one more than the
 * whole number of block lengths in the distance, 1 + floor(d / (4 dx)), with
 * the smallest cell size over the axes; none at B = 1, where every cell sees
 * every face.  n_prop >= 0 overrides the rule. */
static int prop_steps(const orc_forest *fo, int l, int B, int n_prop) {
    if (n_prop >= 0) return n_prop;
    if (B <= 1) return 0;
    float dxm = fo->dx[l][0];
    for (int a = 1; a < fo->dim; ++a) dxm = fmin2(dxm, fo->dx[l][a]);
    return 1 + (int)floorf(fo->d[l] / (4.0f * dxm));
}

static void forest_export(orc_forest *fo) {
    int cells = fo->dim == 3 ? 64 : 16;
    for (int l = 0; l <= fo->L; ++l) {
        orc_level *lv = &fo->lev[l];
        fo->ek[l] = (uint32_t *)xmalloc((size_t)lv->n * sizeof(uint32_t));
        fo->eleaf[l] = (uint8_t *)xmalloc((size_t)lv->n);
        fo->emark[l] = (uint8_t *)xmalloc((size_t)lv->n);
        fo->ecf[l] = (uint8_t *)xmalloc((size_t)lv->n * cells);
        for (int64_t i = 0; i < lv->n; ++i) {
            fo->ek[l][i] = lv->b[i].key;
            fo->eleaf[l][i] = lv->b[i].leaf;
            fo->emark[l][i] = lv->b[i].mark;
            memcpy(fo->ecf[l] + i * cells, lv->b[i].cf, (size_t)cells);
        }
    }
}

/*
 * Level-by-level near-wall refinement.  For pass l = 0..L-1:
 *  (i)   every cell of every block present at level l at the start of the
 *        pass is tested with h = d[l]; the block is flagged (mark 1) when one
 *        of its cells is;
 *  (ii)  ripple for m = l down to 1: for each block of level m marked in this
 *        pass and each of its 3^D - 1 neighbour positions inside the domain
 *        with no level-m block, the covering level-(m-1) leaf is marked
 *        (mark 2, balance);
 *  (iii) every block marked in this pass becomes a parent of 2^D leaf
 *        children one level down (child index x-fastest).
 * Blocks created in pass l are not tested in pass l.
 * bins == NULL selects the brute-force face loop.
 */
static orc_forest *refine_core(int dim, const float *coords, int64_t F, const orc_bins *bn, const int *roots,
                               int L, const float *d_spec, const float *lo, const float *hi, int own_bin,
                               int n_prop) {
    if (L < 0 || L > ORC_MAXL) return NULL;
    if (own_bin && !bn) return NULL;
    orc_forest *fo = (orc_forest *)xcalloc(1, sizeof(orc_forest));
    fo->dim = dim;
    fo->L = L;
    for (int a = 0; a < 3; ++a) {
        fo->roots[a] = a < dim ? roots[a] : 1;
        fo->lo[a] = a < dim ? lo[a] : 0.0f;
        fo->hi[a] = a < dim ? hi[a] : 1.0f;
    }
    for (int l = 0; l <= L; ++l)
        for (int a = 0; a < 3; ++a)
            fo->dx[l][a] = (fo->hi[a] - fo->lo[a]) / (float)(4 * fo->roots[a] * (1 << l));
    for (int l = 0; l < L; ++l) fo->d[l] = d_spec[l];
    int cells = dim == 3 ? 64 : 16;
    int nch = dim == 3 ? 8 : 4;

    /* level 0: all roots */
    for (int z = 0; z < fo->roots[2]; ++z)
        for (int y = 0; y < fo->roots[1]; ++y)
            for (int x = 0; x < fo->roots[0]; ++x) {
                orc_block b;
                memset(&b, 0, sizeof b);
                b.c[0] = x; b.c[1] = y; b.c[2] = z;
                b.key = key_of(fo, 0, b.c);
                b.leaf = 1;
                level_push(&fo->lev[0], &b);
            }
    qsort(fo->lev[0].b, (size_t)fo->lev[0].n, sizeof(orc_block), cmp_block);

    for (int l = 0; l < L; ++l) {
        for (int m = 0; m <= l; ++m)
            for (int64_t i = 0; i < fo->lev[m].n; ++i) fo->lev[m].b[i].pass_mark = 0;
        /* (i) flag */
        orc_level *lv = &fo->lev[l];
        for (int64_t i = 0; i < lv->n; ++i) {
            orc_block *b = &lv->b[i];
            int any = 0;
            for (int c = 0; c < cells; ++c) {
                float m[3] = {0, 0, 0};
                cell_center(fo, l, b->c, c, m);
                b->cf[c] = (uint8_t)(own_bin ? cell_flag_own_bin(fo, coords, bn, m, fo->d[l], &fo->tests[l])
                                             : cell_flag(fo, coords, F, bn, m, fo->d[l], &fo->tests[l]));
                any |= b->cf[c];
            }
            if (any) { b->mark = 1; b->pass_mark = 1; }
        }
        /* (i') own-bin mode: propagation.  Each step first gives every unmarked
         * level-l neighbour (faces, edges, corners) of a marked level-l block
         * an intermediate value, then turns the intermediate values into
         * marks (3 = marked by propagation), so a step grows the marked set by
         * exactly one ring of blocks whatever the visiting order. */
        int nsteps = own_bin ? prop_steps(fo, l, bn->B, n_prop) : 0;
        for (int st = 0; st < nsteps; ++st) {
            for (int64_t i = 0; i < lv->n; ++i) {
                orc_block *b = &lv->b[i];
                if (b->pass_mark != 1 && b->pass_mark != 3) continue;
                for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (!dx && !dy && !dz) continue;
                            int32_t nc[3] = {b->c[0] + dx, b->c[1] + dy, b->c[2] + dz};
                            int inside = 1;
                            for (int a = 0; a < dim; ++a)
                                if (nc[a] < 0 || nc[a] >= fo->roots[a] << l) inside = 0;
                            if (!inside) continue;
                            orc_block *nb = level_find(lv, key_of(fo, l, nc));
                            if (nb && nb->pass_mark == 0) nb->pass_mark = 4;
                        }
            }
            for (int64_t i = 0; i < lv->n; ++i)
                if (lv->b[i].pass_mark == 4) { lv->b[i].pass_mark = 3; lv->b[i].mark = 3; }
        }
        /* (ii) ripple */
        for (int m = l; m >= 1; --m) {
            orc_level *cur = &fo->lev[m];
            for (int64_t i = 0; i < cur->n; ++i) {
                orc_block *b = &cur->b[i];
                if (!b->pass_mark) continue;
                for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (!dx && !dy && !dz) continue;
                            int32_t nc[3] = {b->c[0] + dx, b->c[1] + dy, b->c[2] + dz};
                            int inside = 1;
                            for (int a = 0; a < dim; ++a)
                                if (nc[a] < 0 || nc[a] >= fo->roots[a] << m) inside = 0;
                            if (!inside) continue;
                            if (level_find(cur, key_of(fo, m, nc))) continue;
                            int32_t pc[3] = {nc[0] >> 1, nc[1] >> 1, dim == 3 ? nc[2] >> 1 : 0};
                            orc_block *p = level_find(&fo->lev[m - 1], key_of(fo, m - 1, pc));
                            if (!p || !p->leaf) {
                                fprintf(stderr, "oracle: forest lost 2:1 balance\n");
                                abort();
                            }
                            if (!p->pass_mark) { p->pass_mark = 2; p->mark = 2; }
                        }
            }
        }
        /* (iii) children */
        for (int m = l; m >= 0; --m) {
            orc_level *cur = &fo->lev[m];
            int64_t n0 = cur->n;
            for (int64_t i = 0; i < n0; ++i) {
                orc_block *b = &fo->lev[m].b[i];
                if (!b->pass_mark) continue;
                b->leaf = 0;
                for (int ci = 0; ci < nch; ++ci) {
                    orc_block ch;
                    memset(&ch, 0, sizeof ch);
                    ch.c[0] = 2 * b->c[0] + (ci & 1);
                    ch.c[1] = 2 * b->c[1] + ((ci >> 1) & 1);
                    ch.c[2] = dim == 3 ? 2 * b->c[2] + ((ci >> 2) & 1) : 0;
                    ch.key = b->key * (uint32_t)nch + (uint32_t)ci;
                    ch.leaf = 1;
                    level_push(&fo->lev[m + 1], &ch);
                }
            }
            qsort(fo->lev[m + 1].b, (size_t)fo->lev[m + 1].n, sizeof(orc_block), cmp_block);
        }
    }
    forest_export(fo);
    return fo;
}

orc_forest *orc_refine(int dim, const float *coords, int64_t F, const orc_bins *bn, const int *roots,
                       int L, const float *d_spec, const float *lo, const float *hi) {
    return refine_core(dim, coords, F, bn, roots, L, d_spec, lo, hi, 0, 0);
}

/*
 * The paper's own-bin refinement: as orc_refine, but a cell is flagged when
 * its centre lies within d[l] (Euclidean) of a face of the bin holding the
 * centre, and after the flags each pass propagates its marks to neighbouring
 * level-l blocks, prop_steps() rings of them (mark 3).  Requires bins.
 */
orc_forest *orc_refine_own_bin(int dim, const float *coords, int64_t F, const orc_bins *bn, const int *roots,
                               int L, const float *d_spec, const float *lo, const float *hi, int n_prop) {
    return refine_core(dim, coords, F, bn, roots, L, d_spec, lo, hi, 1, n_prop);
}

void orc_forest_free(orc_forest *fo) {
    if (!fo) return;
    for (int l = 0; l <= ORC_MAXL; ++l) {
        free(fo->lev[l].b); free(fo->ek[l]); free(fo->eleaf[l]); free(fo->emark[l]); free(fo->ecf[l]);
    }
    free(fo);
}
int64_t orc_forest_n(const orc_forest *fo, int l) { return (l < 0 || l > fo->L) ? -1 : fo->lev[l].n; }
const uint32_t *orc_forest_keys(const orc_forest *fo, int l) { return fo->ek[l]; }
const uint8_t *orc_forest_leaf(const orc_forest *fo, int l) { return fo->eleaf[l]; }
const uint8_t *orc_forest_mark(const orc_forest *fo, int l) { return fo->emark[l]; }
const uint8_t *orc_forest_cell_flag(const orc_forest *fo, int l) { return fo->ecf[l]; }
int64_t orc_forest_tests(const orc_forest *fo, int l) { return fo->tests[l]; }

/* ------------------------------------------------------------------ */
/* Link fractions (FP64).                                               */
/* ------------------------------------------------------------------ */
/* Segment o + t*D, t in [0,1], against the closed triangle (a,b,c), two-sided
 * (Moller-Trumbore).  Returns 1 and t, u, v on a hit; det == 0 is no hit. */
static int ray_tri(const double *o, const double *Dv, const double *a, const double *b, const double *c,
                   double *t_out, double *u_out, double *v_out) {
    double E1[3], E2[3], P[3], T[3], Qv[3];
    for (int k = 0; k < 3; ++k) { E1[k] = b[k] - a[k]; E2[k] = c[k] - a[k]; }
    cross3(Dv, E2, P);
    double det = dot3(E1, P);
    if (det == 0.0) return 0;
    for (int k = 0; k < 3; ++k) T[k] = o[k] - a[k];
    double u = dot3(T, P) / det;
    if (u < 0.0 || u > 1.0) return 0;
    cross3(T, E1, Qv);
    double v = dot3(Dv, Qv) / det;
    if (v < 0.0 || u + v > 1.0) return 0;
    double t = dot3(E2, Qv) / det;
    if (t < 0.0 || t > 1.0) return 0;
    *t_out = t; *u_out = u; *v_out = v;
    return 1;
}

/* Segment o + t*D against segment a + s*(b-a), both parameters in [0,1]. */
static int ray_seg(const double *o, const double *Dv, const double *a, const double *b,
                   double *t_out, double *s_out) {
    double e[2] = {b[0] - a[0], b[1] - a[1]};
    double den = Dv[0] * e[1] - Dv[1] * e[0];
    if (den == 0.0) return 0;
    double w[2] = {a[0] - o[0], a[1] - o[1]};
    double t = (w[0] * e[1] - w[1] * e[0]) / den;
    double s = (w[0] * Dv[1] - w[1] * Dv[0]) / den;
    if (t < 0.0 || t > 1.0 || s < 0.0 || s > 1.0) return 0;
    *t_out = t; *s_out = s;
    return 1;
}

/* Hit of the segment with face f: returns 1 and t, plus barycentrics lam[0..dim-1]. */
static int seg_face(int dim, const float *coords, int64_t f, const double *o, const double *Dv,
                    double *t, double *lam) {
    double p[9];
    for (int k = 0; k < dim * dim; ++k) p[k] = (double)coords[f * dim * dim + k];
    if (dim == 3) {
        double u, v;
        if (!ray_tri(o, Dv, p, p + 3, p + 6, t, &u, &v)) return 0;
        lam[0] = 1.0 - u - v; lam[1] = u; lam[2] = v;
        return 1;
    } else {
        double s;
        if (!ray_seg(o, Dv, p, p + 2, t, &s)) return 0;
        lam[0] = 1.0 - s; lam[1] = s;
        return 1;
    }
}

typedef struct {
    int dim, Q;
    int64_t n;
    uint64_t *key;
    double *q;
    int32_t *face;
    int64_t tests;
} orc_links;

static int bin_index_d(double x, double lo, double s, int B) {
    double f = floor((x - lo) * s);
    if (f < 0.0) return 0;
    if (f > (double)(B - 1)) return B - 1;
    return (int)f;
}

/* Candidate faces of a box [blo, bhi] from the bins (FP64 index, conservative). */
typedef struct { int32_t *f; int64_t n, cap; } idlist;
static void idlist_push(idlist *L, int32_t f) {
    if (L->n == L->cap) { L->cap = L->cap ? 2 * L->cap : 256; L->f = (int32_t *)xrealloc(L->f, (size_t)L->cap * 4); }
    L->f[L->n++] = f;
}
static void box_candidates(const orc_bins *bn, int dim, int64_t F, const double *blo, const double *bhi, idlist *out) {
    out->n = 0;
    if (!bn) { for (int64_t f = 0; f < F; ++f) idlist_push(out, (int32_t)f); return; }
    int l[3] = {0, 0, 0}, u[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        double s = (double)bn->B / ((double)bn->hi[a] - (double)bn->lo[a]);
        l[a] = bin_index_d(blo[a], bn->lo[a], s, bn->B);
        u[a] = bin_index_d(bhi[a], bn->lo[a], s, bn->B);
    }
    int B = bn->B;
    for (int z = l[2]; z <= u[2]; ++z)
        for (int y = l[1]; y <= u[1]; ++y)
            for (int x = l[0]; x <= u[0]; ++x) {
                int64_t b = ((int64_t)z * B + y) * B + x;
                for (uint32_t j = bn->off[b]; j < bn->off[b + 1]; ++j) idlist_push(out, bn->ids[j]);
            }
}

/* q for one cell: fills q[Q], face[Q]; returns the number of links. */
static int cell_links(int dim, int Q, const int *cv, const float *coords, int64_t F, const orc_bins *bn,
                      const double *o, const double *dxL, idlist *cand, double *q, int32_t *face, int64_t *ntests) {
    double blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
    const double eps = 9.5367431640625e-07;
    for (int a = 0; a < dim; ++a) { blo[a] = o[a] - dxL[a] - eps; bhi[a] = o[a] + dxL[a] + eps; }
    box_candidates(bn, dim, F, blo, bhi, cand);
    *ntests += cand->n;
    int nl = 0;
    q[0] = -1.0; face[0] = -1;
    for (int i = 1; i < Q; ++i) {
        double Dv[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) Dv[a] = (double)cv[3 * i + a] * dxL[a];
        double best = INFINITY;
        int32_t bf = -1;
        for (int64_t j = 0; j < cand->n; ++j) {
            int32_t f = cand->f[j];
            double t, lam[3];
            if (!seg_face(dim, coords, f, o, Dv, &t, lam)) continue;
            if (t < best || (t == best && f < bf)) { best = t; bf = f; }
        }
        if (bf >= 0) { q[i] = best; face[i] = bf; ++nl; }
        else { q[i] = -1.0; face[i] = -1; }
    }
    return nl;
}

/*
 * Link fractions at the finest level L of the forest: for every cell of
 * every level-L block (all of them, or the block indices in `subset`) and
 * every non-rest direction c_i, q_i is the smallest t in [0,1] at which
 * x + t c_i dx_L meets a face, face_i the lowest face id attaining it
 * (-1/-1 when none).  Cells with at least one link are emitted in
 * canonical order (block key, then cell x-fastest) with node key
 * block_key * 4^D + cell.  bins == NULL selects every face as a candidate.
 */
orc_links *orc_link_fractions(int dim, const float *coords, int64_t F, const orc_bins *bn,
                              const orc_forest *fo, int Q, const int64_t *subset, int64_t n_subset) {
    int cv[27 * 3];
    if (orc_lattice(Q, cv) != dim) return NULL;
    int L = fo->L;
    int cells = dim == 3 ? 64 : 16;
    const orc_level *lv = &fo->lev[L];
    int64_t nblk = subset ? n_subset : lv->n;
    orc_links *lk = (orc_links *)xcalloc(1, sizeof(orc_links));
    lk->dim = dim; lk->Q = Q;
    int64_t cap = 1024;
    lk->key = (uint64_t *)xmalloc((size_t)cap * 8);
    lk->q = (double *)xmalloc((size_t)cap * Q * 8);
    lk->face = (int32_t *)xmalloc((size_t)cap * Q * 4);
    double dxL[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) dxL[a] = (double)fo->dx[L][a];
    idlist cand = {0, 0, 0};
    double q[27];
    int32_t fc[27];
    for (int64_t bi = 0; bi < nblk; ++bi) {
        int64_t i = subset ? subset[bi] : bi;
        const orc_block *b = &lv->b[i];
        for (int c = 0; c < cells; ++c) {
            float m[3] = {0, 0, 0};
            cell_center(fo, L, b->c, c, m);
            double o[3] = {m[0], m[1], m[2]};
            if (!cell_links(dim, Q, cv, coords, F, bn, o, dxL, &cand, q, fc, &lk->tests)) continue;
            if (lk->n == cap) {
                cap *= 2;
                lk->key = (uint64_t *)xrealloc(lk->key, (size_t)cap * 8);
                lk->q = (double *)xrealloc(lk->q, (size_t)cap * Q * 8);
                lk->face = (int32_t *)xrealloc(lk->face, (size_t)cap * Q * 4);
            }
            lk->key[lk->n] = (uint64_t)b->key * (uint64_t)cells + (uint64_t)c;
            memcpy(lk->q + lk->n * Q, q, (size_t)Q * 8);
            memcpy(lk->face + lk->n * Q, fc, (size_t)Q * 4);
            lk->n++;
        }
    }
    free(cand.f);
    return lk;
}

void orc_links_free(orc_links *lk) {
    if (!lk) return;
    free(lk->key); free(lk->q); free(lk->face); free(lk);
}
int64_t orc_links_n(const orc_links *lk) { return lk->n; }
const uint64_t *orc_links_key(const orc_links *lk) { return lk->key; }
const double *orc_links_q(const orc_links *lk) { return lk->q; }
const int32_t *orc_links_face(const orc_links *lk) { return lk->face; }
int64_t orc_links_tests(const orc_links *lk) { return lk->tests; }

/* Node key -> cell centre (FP32 rule, promoted) for a node of level L. */
static void node_origin(const orc_forest *fo, uint64_t nkey, double *o) {
    int dim = fo->dim, L = fo->L;
    int cells = dim == 3 ? 64 : 16, nch = dim == 3 ? 8 : 4;
    uint32_t key = (uint32_t)(nkey / (uint64_t)cells);
    int cell = (int)(nkey % (uint64_t)cells);
    /* decode block coordinates from the hierarchical key */
    uint32_t k = key;
    int32_t path[3] = {0, 0, 0};
    for (int j = 0; j < L; ++j) {
        uint32_t ci = k % (uint32_t)nch;
        k /= (uint32_t)nch;
        path[0] |= (int32_t)(ci & 1) << j;
        path[1] |= (int32_t)((ci >> 1) & 1) << j;
        if (dim == 3) path[2] |= (int32_t)((ci >> 2) & 1) << j;
    }
    int32_t r0 = (int32_t)(k % (uint32_t)fo->roots[0]);
    int32_t r1 = (int32_t)((k / (uint32_t)fo->roots[0]) % (uint32_t)fo->roots[1]);
    int32_t r2 = (int32_t)(k / ((uint32_t)fo->roots[0] * (uint32_t)fo->roots[1]));
    int32_t bc[3] = {(r0 << L) | path[0], (r1 << L) | path[1], dim == 3 ? ((r2 << L) | path[2]) : 0};
    float m[3] = {0, 0, 0};
    cell_center(fo, L, bc, cell, m);
    o[0] = m[0]; o[1] = m[1]; o[2] = m[2];
}

/* ------------------------------------------------------------------ */
/* Adjoint (FP64): for L = sum_i w_i q_i over link slots,               */
/*   dL/dv_k += w_i * lambda_k * n / (Dv . n)                           */
/* for the hit face's vertex k (n a face normal, lambda the barycentric */
/* weights of the hit), accumulated onto unique vertices.               */
/* ------------------------------------------------------------------ */
static void face_normal(int dim, const double *p, double *n) {
    if (dim == 3) {
        double e1[3], e2[3];
        for (int a = 0; a < 3; ++a) { e1[a] = p[3 + a] - p[a]; e2[a] = p[6 + a] - p[a]; }
        cross3(e1, e2, n);
    } else {
        n[0] = -(p[3] - p[1]);
        n[1] = p[2] - p[0];
        n[2] = 0.0;
    }
}

/*
 * Re-adaptation bookkeeping (the refine-and-coarsen step that a moving body
 * needs each time its geometry changes; the paper refines only once, before
 * the solver, and names moving geometry as the case to come, Results
 * discussion).  The re-adapted forest itself is the near-wall refinement of
 * the new geometry; what a solver also needs is how it relates to the old
 * forest, level by level, over the same root grid.  Per block of the new
 * level: old_index = its position in the old level (-1: absent) and state
 *   0 kept (present in both with the same leaf bit),
 *   1 created (absent from the old level),
 *   2 refined (a leaf before, now with children),
 *   3 coarsened (children before, now a leaf: its children are removed);
 * per block of the old level: removed = 1 when its key is absent from the new
 * level.  Keys of a level are sorted ascending; each lookup is a binary search.
 */
static int64_t key_search(const uint32_t *keys, int64_t n, uint32_t k) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == k) return mid;
        if (keys[mid] < k) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

void orc_forest_diff(const uint32_t *old_keys, const uint8_t *old_leaf, int64_t n_old, const uint32_t *new_keys,
                     const uint8_t *new_leaf, int64_t n_new, int32_t *old_index, uint8_t *state,
                     uint8_t *removed) {
    for (int64_t i = 0; i < n_new; ++i) {
        int64_t j = key_search(old_keys, n_old, new_keys[i]);
        old_index[i] = (int32_t)j;
        if (j < 0) state[i] = 1;
        else if (old_leaf[j] && !new_leaf[i]) state[i] = 2;
        else if (!old_leaf[j] && new_leaf[i]) state[i] = 3;
        else state[i] = 0;
    }
    for (int64_t j = 0; j < n_old; ++j) removed[j] = key_search(new_keys, n_new, old_keys[j]) < 0 ? 1 : 0;
}

/*
 * Node classification: the step after the link fractions that the paper
 * leaves to future work (Results discussion, Conclusion).  With the faces
 * oriented so that n = (b - a) x (c - a) (3D) or n = (e_y, -e_x), e = b - a
 * (2D) points out of the solid, a link from a node outside the solid first
 * meets a face it enters (c_i . n < 0), a link from a node inside first meets
 * a face it leaves (c_i . n > 0).  Per node: 1 (fluid) when every link
 * enters, 2 (solid) when every link leaves, 3 when its links disagree.
 * s_i = (c_i0 n0 + c_i1 n1) + c_i2 n2 in FP64, n from the face's FP32 corners
 * (components a1 b2 - a2 b1, a2 b0 - a0 b2, a0 b1 - a1 b0).
 *   face: n_nodes x Q face ids (-1 = no link), coords: F x dim x dim.
 */
void orc_classify_nodes(int dim, int Q, int64_t n_nodes, const int32_t *face, const float *coords, uint8_t *cls) {
    int c[27 * 3];
    orc_lattice(Q, c);
    for (int64_t k = 0; k < n_nodes; ++k) {
        int enter = 0, leave = 0;
        for (int i = 1; i < Q; ++i) {
            int32_t f = face[k * Q + i];
            if (f < 0) continue;
            const float *v = coords + (int64_t)f * dim * dim;
            double nrm[3] = {0, 0, 0};
            if (dim == 3) {
                double e1[3], e2[3];
                for (int a = 0; a < 3; ++a) {
                    e1[a] = (double)v[3 + a] - (double)v[a];
                    e2[a] = (double)v[6 + a] - (double)v[a];
                }
                nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
                nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
                nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
            } else {
                double e0 = (double)v[2] - (double)v[0], e1 = (double)v[3] - (double)v[1];
                nrm[0] = e1;
                nrm[1] = -e0;
            }
            double sgn = ((double)c[3 * i] * nrm[0] + (double)c[3 * i + 1] * nrm[1]) + (double)c[3 * i + 2] * nrm[2];
            if (sgn < 0.0) enter = 1;
            else if (sgn > 0.0) leave = 1;
            else { enter = 1; leave = 1; }   /* a hit along the face's plane has no side */
        }
        cls[k] = (uint8_t)(enter && leave ? 3 : (leave ? 2 : 1));
    }
}

void orc_link_grad(const orc_forest *fo, const orc_links *lk, const float *coords, const int32_t *fidx,
                   const double *w, double *grad) {
    int dim = lk->dim, Q = lk->Q;
    int cv[27 * 3];
    orc_lattice(Q, cv);
    double dxL[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) dxL[a] = (double)fo->dx[fo->L][a];
    for (int64_t n = 0; n < lk->n; ++n) {
        double o[3];
        node_origin(fo, lk->key[n], o);
        for (int i = 1; i < Q; ++i) {
            double wi = w[n * Q + i];
            int32_t f = lk->face[n * Q + i];
            if (f < 0 || wi == 0.0) continue;
            double Dv[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) Dv[a] = (double)cv[3 * i + a] * dxL[a];
            double t, lam[3];
            if (!seg_face(dim, coords, f, o, Dv, &t, lam)) continue;
            double p[9] = {0}, nrm[3];
            for (int k = 0; k < dim * dim; ++k) p[k] = (double)coords[(int64_t)f * dim * dim + k];
            face_normal(dim, p, nrm);
            double den = 0.0;
            for (int a = 0; a < dim; ++a) den += Dv[a] * nrm[a];
            for (int k = 0; k < dim; ++k) {
                int64_t vk = fidx[(int64_t)f * dim + k];
                for (int a = 0; a < dim; ++a) grad[vk * dim + a] += wi * lam[k] * nrm[a] / den;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Stability screen for finite differences: a link slot is kept when   */
/*  eta = h / (alt_min * |cos theta|) <= eta_max, every barycentric of  */
/*  the hit >= bary_min, t in [t_lo, 1 - t_lo], and no other candidate  */
/*  face hits within gap in t.                                          */
/* ------------------------------------------------------------------ */
void orc_link_stable(const orc_forest *fo, const orc_links *lk, const float *coords, int64_t F,
                     const orc_bins *bn, double h, double eta_max, double bary_min, double t_lo,
                     double gap, uint8_t *stable) {
    int dim = lk->dim, Q = lk->Q;
    int cv[27 * 3];
    orc_lattice(Q, cv);
    double dxL[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) dxL[a] = (double)fo->dx[fo->L][a];
    idlist cand = {0, 0, 0};
    const double eps = 9.5367431640625e-07;
    for (int64_t n = 0; n < lk->n; ++n) {
        double o[3];
        node_origin(fo, lk->key[n], o);
        double blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) { blo[a] = o[a] - dxL[a] - eps - h; bhi[a] = o[a] + dxL[a] + eps + h; }
        box_candidates(bn, dim, F, blo, bhi, &cand);
        for (int i = 0; i < Q; ++i) {
            uint8_t ok = 0;
            int32_t f = lk->face[n * Q + i];
            if (i > 0 && f >= 0) {
                double Dv[3] = {0, 0, 0};
                for (int a = 0; a < dim; ++a) Dv[a] = (double)cv[3 * i + a] * dxL[a];
                double t, lam[3];
                if (seg_face(dim, coords, f, o, Dv, &t, lam)) {
                    double p[9] = {0}, nrm[3];
                    for (int k = 0; k < dim * dim; ++k) p[k] = (double)coords[(int64_t)f * dim * dim + k];
                    face_normal(dim, p, nrm);
                    double nn = 0.0, dd = 0.0, dn = 0.0;
                    for (int a = 0; a < dim; ++a) { nn += nrm[a] * nrm[a]; dd += Dv[a] * Dv[a]; dn += Dv[a] * nrm[a]; }
                    double emax = 0.0;
                    for (int k = 0; k < dim; ++k) {
                        int k2 = (k + 1) % dim;
                        double e2 = 0.0;
                        for (int a = 0; a < dim; ++a) { double d = p[k2 * dim + a] - p[k * dim + a]; e2 += d * d; }
                        if (e2 > emax) emax = e2;
                    }
                    /* minimum altitude: 2*area / longest edge (3D); segment length (2D) */
                    double alt = dim == 3 ? sqrt(nn) / sqrt(emax) : sqrt(emax);
                    double cosv = fabs(dn) / sqrt(nn * dd);
                    double eta = (cosv > 0.0 && alt > 0.0) ? h / (alt * cosv) : INFINITY;
                    double lmin = lam[0];
                    for (int k = 1; k < dim; ++k) if (lam[k] < lmin) lmin = lam[k];
                    ok = eta <= eta_max && lmin >= bary_min && t >= t_lo && t <= 1.0 - t_lo;
                    if (ok) {
                        for (int64_t j = 0; j < cand.n && ok; ++j) {
                            int32_t g = cand.f[j];
                            if (g == f) continue;
                            double t2, lam2[3];
                            if (seg_face(dim, coords, g, o, Dv, &t2, lam2) && fabs(t2 - t) < gap) ok = 0;
                        }
                    }
                }
            }
            stable[n * Q + i] = ok;
        }
    }
    free(cand.f);
}

/* ------------------------------------------------------------------ */
/* Central finite differences of L = sum w_i q_i with respect to each   */
/* coordinate of the listed vertices (FP64), step h.  Only link slots   */
/* whose candidate set (bins over the link box widened by h) holds a    */
/* face incident to the vertex are recomputed, each by a full minimum   */
/* over its candidates with the perturbed coordinates.  Slots whose     */
/* arg-min face changes at +h or -h are counted in *n_changed.          */
/* ------------------------------------------------------------------ */
void orc_fd_grad(const orc_forest *fo, const orc_links *lk, const float *verts, int64_t Nv,
                 const int32_t *fidx, int64_t F, const orc_bins *bn, const double *w, double h,
                 const int64_t *vsub, int64_t n_vsub, double *grad_fd, int64_t *n_changed) {
    int dim = lk->dim, Q = lk->Q;
    int cv[27 * 3];
    orc_lattice(Q, cv);
    double dxL[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) dxL[a] = (double)fo->dx[fo->L][a];
    const double eps = 9.5367431640625e-07;
    /* FP64 working copy of the vertices */
    double *V = (double *)xmalloc((size_t)Nv * dim * 8);
    for (int64_t i = 0; i < Nv * dim; ++i) V[i] = (double)verts[i];
    /* FP32 coordinate list for the bin lookup (unperturbed) */
    /* incidence: vertex -> link nodes whose candidate set contains an incident face */
    int64_t *cnt = (int64_t *)xcalloc((size_t)Nv + 1, 8);
    idlist cand = {0, 0, 0};
    float *coords = (float *)xmalloc((size_t)F * dim * dim * 4);
    orc_gather(dim, verts, fidx, F, coords);
    /* node -> candidate list cache */
    int64_t *coff = (int64_t *)xcalloc((size_t)lk->n + 1, 8);
    idlist all = {0, 0, 0};
    for (int64_t n = 0; n < lk->n; ++n) {
        int any = 0;
        for (int i = 1; i < Q; ++i) if (w[n * Q + i] != 0.0 && lk->face[n * Q + i] >= 0) any = 1;
        coff[n] = all.n;
        if (!any) continue;
        double o[3];
        node_origin(fo, lk->key[n], o);
        double blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) { blo[a] = o[a] - dxL[a] - eps - h; bhi[a] = o[a] + dxL[a] + eps + h; }
        box_candidates(bn, dim, F, blo, bhi, &cand);
        for (int64_t j = 0; j < cand.n; ++j) idlist_push(&all, cand.f[j]);
    }
    coff[lk->n] = all.n;
    /* vertex -> nodes (with duplicates removed per vertex via a stamp) */
    int64_t *stamp = (int64_t *)xmalloc((size_t)Nv * 8);
    for (int64_t i = 0; i < Nv; ++i) stamp[i] = -1;
    for (int64_t n = 0; n < lk->n; ++n)
        for (int64_t j = coff[n]; j < coff[n + 1]; ++j)
            for (int k = 0; k < dim; ++k) {
                int64_t vk = fidx[(int64_t)all.f[j] * dim + k];
                if (stamp[vk] != n) { stamp[vk] = n; cnt[vk + 1]++; }
            }
    for (int64_t i = 0; i < Nv; ++i) cnt[i + 1] += cnt[i];
    int64_t *vn = (int64_t *)xmalloc((size_t)cnt[Nv] * 8 + 8);
    int64_t *fill = (int64_t *)xcalloc((size_t)Nv, 8);
    for (int64_t i = 0; i < Nv; ++i) stamp[i] = -1;
    for (int64_t n = 0; n < lk->n; ++n)
        for (int64_t j = coff[n]; j < coff[n + 1]; ++j)
            for (int k = 0; k < dim; ++k) {
                int64_t vk = fidx[(int64_t)all.f[j] * dim + k];
                if (stamp[vk] != n) { stamp[vk] = n; vn[cnt[vk] + fill[vk]++] = n; }
            }
    *n_changed = 0;
    for (int64_t si = 0; si < n_vsub; ++si) {
        int64_t vk = vsub[si];
        for (int a = 0; a < dim; ++a) {
            double Lpm[2] = {0.0, 0.0};
            for (int sgn = 0; sgn < 2; ++sgn) {
                double save = V[vk * dim + a];
                V[vk * dim + a] = save + (sgn == 0 ? h : -h);
                for (int64_t r = cnt[vk]; r < cnt[vk + 1]; ++r) {
                    int64_t n = vn[r];
                    double o[3];
                    node_origin(fo, lk->key[n], o);
                    for (int i = 1; i < Q; ++i) {
                        double wi = w[n * Q + i];
                        if (wi == 0.0 || lk->face[n * Q + i] < 0) continue;
                        double Dv[3] = {0, 0, 0};
                        for (int b = 0; b < dim; ++b) Dv[b] = (double)cv[3 * i + b] * dxL[b];
                        double best = INFINITY;
                        int32_t bf = -1;
                        for (int64_t j = coff[n]; j < coff[n + 1]; ++j) {
                            int32_t f = all.f[j];
                            double p[9];
                            for (int k = 0; k < dim; ++k)
                                for (int b = 0; b < dim; ++b) p[k * dim + b] = V[(int64_t)fidx[(int64_t)f * dim + k] * dim + b];
                            double t, u, v, s;
                            int hit = dim == 3 ? ray_tri(o, Dv, p, p + 3, p + 6, &t, &u, &v)
                                               : ray_seg(o, Dv, p, p + 2, &t, &s);
                            if (hit && (t < best || (t == best && f < bf))) { best = t; bf = f; }
                        }
                        if (bf != lk->face[n * Q + i]) { (*n_changed)++; continue; }
                        Lpm[sgn] += wi * (best - lk->q[n * Q + i]);
                    }
                }
                V[vk * dim + a] = save;
            }
            grad_fd[vk * dim + a] = (Lpm[0] - Lpm[1]) / (2.0 * h);
        }
    }
    free(V); free(cnt); free(cand.f); free(coords); free(coff); free(all.f); free(stamp); free(vn); free(fill);
}

/* t of the link (node, direction i) against one given face f, FP64; returns 1
 * on a hit.  Used to check that a face reported for a link is a hit at the
 * reported fraction (ties between faces sharing an edge or vertex). */
int orc_link_t(const orc_forest *fo, uint64_t node_key, int Q, int i, const float *coords, int32_t f, double *t) {
    int cv[27 * 3];
    int dim = fo->dim;
    if (orc_lattice(Q, cv) != dim || i <= 0 || i >= Q) return 0;
    double o[3], Dv[3] = {0, 0, 0}, lam[3];
    node_origin(fo, node_key, o);
    for (int a = 0; a < dim; ++a) Dv[a] = (double)cv[3 * i + a] * (double)fo->dx[fo->L][a];
    return seg_face(dim, coords, f, o, Dv, t, lam);
}
