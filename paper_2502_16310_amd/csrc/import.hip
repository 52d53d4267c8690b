// Import (paper Sec. II-B): index lists or a coordinate list -> the
// library-owned structure-of-arrays coordinate list, per-face bounding
// boxes, one 16/8-float record per face (corners and box, for single-line
// gathers) and a copy of the index list (needed by the adjoint).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "agal_internal.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace agal {

// Validate and gather in one pass.  err bit 0: a non-finite vertex
// coordinate; bit 1: a face index outside [0, Nv) (such a face is written as
// zeros and the call fails).
template <int D>
__global__ void k_import(const float *verts, int64_t Nv, const int32_t *faces, int64_t F, float *coords, float *aabb,
                         float *rec, int32_t *fidx, uint32_t *acc) {
    uint32_t bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < Nv * D; i += stride)
        if (!isfinite(verts[i])) bad |= 1u;
    float ext[D] = {};
    for (int64_t f = t0; f < F; f += stride)
        bad |= kern::import_face<D>(verts, Nv, faces, F, coords, aabb, rec, fidx, f, ext);
    // error bits in device words (acc[3], acc[4]), zero before the launch
    if (bad & 1u) atomicOr(acc + 3, 1u);
    if (bad & 2u) atomicOr(acc + 4, 1u);
    // largest face box extent per axis: wave maximum, one atomic per wave on
    // the (non-negative) float bits in acc[0 .. D)
#pragma unroll
    for (int a = 0; a < D; ++a) {
        float e = ext[a];
#pragma unroll
        for (int d = dev::kWave / 2; d >= 1; d >>= 1) e = fmaxf(e, __shfl_xor(e, d, dev::kWave));
        if (dev::lane_id() == 0) atomicMax(acc + a, __float_as_uint(e));
    }
}

// After the import kernel (stream order makes its device words final): the
// error bits to err[0..1] and the extents to err[2..2+D) of mapped host
// memory, the device words cleared, then the completion signal.
__global__ void k_import_signal(uint32_t *acc, uint32_t *err, int D, HostSignal sig) {
    if (threadIdx.x != 0) return;
    err[0] = acc[3];
    err[1] = acc[4];
    for (int a = 0; a < D; ++a) err[2 + a] = acc[a];
    for (int i = 0; i < 5; ++i) acc[i] = 0u;
    dev::publish_host(sig.word, sig.seq);
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

    auto *g = new (std::nothrow) agal_geom_t();
    if (!g) return fail(AGAL_ENOMEM, "agal_import_faces: host allocation failed");
    g->ctx = ctx;
    g->id = next_handle_id();
    g->stream = s;
    g->dim = dim;
    g->F = n_faces;
    g->Nv = n_vertices;
    agal_status st = dev_alloc(ctx->mem, &g->coords, (size_t)dim * dim * n_faces, s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &g->aabb, (size_t)2 * dim * n_faces, s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &g->rec, (size_t)(dim == 3 ? 16 : 8) * n_faces, s);
    if (st == AGAL_OK) st = dev_alloc(ctx->mem, &g->fidx, (size_t)dim * n_faces, s);
    if (st != AGAL_OK) {
        agal_destroy_geom(g);
        return st;
    }
    // error words in the context's mapped host memory (no kernel of an earlier
    // call still writes them: every call that uses them synchronises)
    uint32_t *err = ctx->d_counts;
    ctx->h_counts[0] = 0u;
    ctx->h_counts[1] = 0u;
    const HostSignal sig = host_signal(ctx);
    {
        ProfScope prof(ctx, "import", s);
        const unsigned grid = grid_for(std::max(n_vertices * dim, n_faces));
        if (dim == 3)
            hipLaunchKernelGGL(k_import<3>, dim3(grid), dim3(256), 0, s, d_vertices, n_vertices, d_faces, n_faces,
                               g->coords, g->aabb, g->rec, g->fidx, ctx->d_done + 1);
        else
            hipLaunchKernelGGL(k_import<2>, dim3(grid), dim3(256), 0, s, d_vertices, n_vertices, d_faces, n_faces,
                               g->coords, g->aabb, g->rec, g->fidx, ctx->d_done + 1);
        hipLaunchKernelGGL(k_import_signal, dim3(1), dim3(64), 0, s, ctx->d_done + 1, err, dim, sig);
    }
    hipError_t e = hipGetLastError();
    st = e != hipSuccess ? fail(AGAL_EHIP, "agal_import_faces: %s", hipGetErrorString(e))
                         : wait_signal(ctx, s, sig, "agal_import_faces");
    const uint32_t herr = (ctx->h_counts[0] ? 1u : 0u) | (ctx->h_counts[1] ? 2u : 0u);
    for (int a = 0; a < 3; ++a) {
        uint32_t bits = a < dim ? ctx->h_counts[2 + a] : 0u;
        float e;
        std::memcpy(&e, &bits, sizeof e);
        g->max_extent[a] = e;
    }
    if (st == AGAL_OK && (herr & 1u)) st = fail(AGAL_EINVAL, "agal_import_faces: NaN or Inf vertex coordinate");
    if (st == AGAL_OK && (herr & 2u)) st = fail(AGAL_EINVAL, "agal_import_faces: face index outside [0, n_vertices)");
    if (st != AGAL_OK) {
        agal_destroy_geom(g);
        return st;
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
    dev_free(g->ctx->mem, g->rec, g->stream);
    dev_free(g->ctx->mem, g->fidx, g->stream);
    delete g;
}

}  // extern "C"
