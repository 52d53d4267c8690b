// Import (paper Sec. II-B): index lists or a coordinate list -> the
// library-owned structure-of-arrays coordinate list, per-face bounding
// boxes and a copy of the index list (needed by the adjoint).
#include <algorithm>
#include <cmath>

#include "agal_internal.hpp"
#include "device.hpp"

namespace agal {

// bit 0: non-finite coordinate, bit 1: index out of range
__global__ void k_import_check(const float *verts, int64_t nvc, const int32_t *faces, int64_t nfi, int64_t Nv,
                               uint32_t *err) {
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvc; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(verts[i])) bad |= 1u;
    if (faces)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nfi; i += (int64_t)gridDim.x * blockDim.x) {
            int32_t v = faces[i];
            if (v < 0 || (int64_t)v >= Nv) bad |= 2u;
        }
    if (bad) atomicOr(err, bad);
}

template <int D>
__global__ void k_import_gather(const float *verts, const int32_t *faces, int64_t F, float *coords, float *aabb,
                                int32_t *fidx) {
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
        float v[D][D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            int64_t vi = faces ? (int64_t)faces[f * D + k] : f * D + k;
            fidx[f * D + k] = (int32_t)vi;
#pragma unroll
            for (int a = 0; a < D; ++a) v[k][a] = verts[vi * D + a];
        }
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
            for (int a = 0; a < D; ++a) coords[(int64_t)(k * D + a) * F + f] = v[k][a];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            float mn = v[0][a], mx = v[0][a];
#pragma unroll
            for (int k = 1; k < D; ++k) {
                mn = dev::fminf_(mn, v[k][a]);
                mx = dev::fmaxf_(mx, v[k][a]);
            }
            aabb[(int64_t)a * F + f] = mn;
            aabb[(int64_t)(D + a) * F + f] = mx;
        }
    }
}

static unsigned grid_for(int64_t n, int threads = 256, int64_t cap = 8192) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace agal

using namespace agal;

extern "C" {

agal_status agal_import_faces(agal_context ctx, int dim, const float *d_vertices, int64_t n_vertices,
                              const int32_t *d_faces, int64_t n_faces, void *stream, agal_geom *out) {
    if (!ctx || !out) return fail(AGAL_EINVAL, "agal_import_faces: NULL context or out");
    if (dim != 2 && dim != 3) return fail(AGAL_EINVAL, "agal_import_faces: dim must be 2 or 3 (got %d)", dim);
    if (n_faces < 1 || n_vertices < 1) return fail(AGAL_EINVAL, "agal_import_faces: empty geometry");
    if (n_faces > (int64_t)INT32_MAX) return fail(AGAL_EINVAL, "agal_import_faces: more than 2^31-1 faces");
    if (!d_vertices) return fail(AGAL_EINVAL, "agal_import_faces: d_vertices is NULL");
    if (!d_faces && n_vertices != n_faces * dim)
        return fail(AGAL_EINVAL, "agal_import_faces: a coordinate list needs n_vertices == n_faces * dim");
    hipStream_t s = (hipStream_t)stream;

    // validate on the device before any gather touches the indices
    uint32_t *err = nullptr;
    AGAL_TRY(dev_alloc(ctx->mem, &err, 1, s));
    fill_u32(err, 0u, 1, s);
    ProfScope prof_check(ctx, "import_check", s);
    hipLaunchKernelGGL(k_import_check, dim3(grid_for(std::max(n_vertices * dim, n_faces * dim))), dim3(256), 0, s,
                       d_vertices, n_vertices * dim, d_faces, n_faces * dim, n_vertices, err);
    uint32_t herr = 0;
    const uint32_t *srcs[1] = {err};
    agal_status st = read_back_u32(ctx, srcs, 1, &herr, s);
    dev_free(ctx->mem, err, s);
    AGAL_TRY(st);
    if (herr & 1u) return fail(AGAL_EINVAL, "agal_import_faces: NaN or Inf vertex coordinate");
    if (herr & 2u) return fail(AGAL_EINVAL, "agal_import_faces: face index outside [0, n_vertices)");

    auto *g = new (std::nothrow) agal_geom_t();
    if (!g) return fail(AGAL_ENOMEM, "agal_import_faces: host allocation failed");
    g->ctx = ctx;
    g->id = next_handle_id();
    g->stream = s;
    g->dim = dim;
    g->F = n_faces;
    g->Nv = n_vertices;
    agal_status a1 = dev_alloc(ctx->mem, &g->coords, (size_t)dim * dim * n_faces, s);
    agal_status a2 = a1 == AGAL_OK ? dev_alloc(ctx->mem, &g->aabb, (size_t)2 * dim * n_faces, s) : a1;
    agal_status a3 = a2 == AGAL_OK ? dev_alloc(ctx->mem, &g->fidx, (size_t)dim * n_faces, s) : a2;
    if (a3 != AGAL_OK) {
        agal_destroy_geom(g);
        return a3;
    }
    ProfScope prof_gather(ctx, "import_gather", s);
    if (dim == 3)
        hipLaunchKernelGGL(k_import_gather<3>, dim3(grid_for(n_faces)), dim3(256), 0, s, d_vertices, d_faces, n_faces,
                           g->coords, g->aabb, g->fidx);
    else
        hipLaunchKernelGGL(k_import_gather<2>, dim3(grid_for(n_faces)), dim3(256), 0, s, d_vertices, d_faces, n_faces,
                           g->coords, g->aabb, g->fidx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        agal_destroy_geom(g);
        return fail(AGAL_EHIP, "agal_import_faces: launch failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return AGAL_OK;
}

agal_status agal_geom_view(agal_geom g, int *dim, int64_t *n_faces, int64_t *n_vertices, const float **d_coords,
                           const float **d_aabb) {
    if (!g) return fail(AGAL_EINVAL, "agal_geom_view: NULL geometry");
    if (dim) *dim = g->dim;
    if (n_faces) *n_faces = g->F;
    if (n_vertices) *n_vertices = g->Nv;
    if (d_coords) *d_coords = g->coords;
    if (d_aabb) *d_aabb = g->aabb;
    return AGAL_OK;
}

void agal_destroy_geom(agal_geom g) {
    if (!g) return;
    dev_free(g->ctx->mem, g->coords, g->stream);
    dev_free(g->ctx->mem, g->aabb, g->stream);
    dev_free(g->ctx->mem, g->fidx, g->stream);
    delete g;
}

}  // extern "C"
