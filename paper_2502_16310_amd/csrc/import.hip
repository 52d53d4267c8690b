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

// Validate and gather in one pass.  Each workgroup reduces its error bits
// (bit 0: a non-finite vertex coordinate; bit 1: a face index outside
// [0, Nv), such a face is written as zeros and the call fails) and its
// largest face box extent per axis, and stores them in its own four words
// part[4 b .. 4 b + 3] (extents as float bits, then the error bits): no
// atomics, which would serialise thousands of workgroups on three addresses.
template <int D>
__global__ __launch_bounds__(256) void k_import(const float *verts, int64_t Nv, const int32_t *faces, int64_t F,
                                                float *coords, float *aabb, float *rec, int32_t *fidx,
                                                uint32_t *part) {
    __shared__ uint32_t s_red[4][256 / dev::kWave];
    uint32_t bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < Nv * D; i += stride)
        if (!isfinite(verts[i])) bad |= 1u;
    float ext[D] = {};
    for (int64_t f = t0; f < F; f += stride)
        bad |= kern::import_face<D>(verts, Nv, faces, F, coords, aabb, rec, fidx, f, ext);
    const int w = threadIdx.x / dev::kWave;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        float e = ext[a];
#pragma unroll
        for (int d = dev::kWave / 2; d >= 1; d >>= 1) e = fmaxf(e, __shfl_xor(e, d, dev::kWave));
        if (dev::lane_id() == 0) s_red[a][w] = __float_as_uint(e);
    }
    const uint64_t b1 = __ballot((bad & 1u) != 0), b2 = __ballot((bad & 2u) != 0);
    if (dev::lane_id() == 0) s_red[3][w] = (b1 ? 1u : 0u) | (b2 ? 2u : 0u);
    __syncthreads();
    if (threadIdx.x < 4) {
        uint32_t r = 0;
        for (int j = 0; j < 256 / dev::kWave; ++j)
            r = threadIdx.x == 3 ? (r | s_red[3][j]) : (threadIdx.x < D ? max(r, s_red[threadIdx.x][j]) : 0u);
        part[4 * (int64_t)blockIdx.x + threadIdx.x] = r;
    }
}

// After the import kernel (stream order makes its partial words final): the
// error bits to err[0..1] and the extents (non-negative float bits, so they
// order as unsigned) to err[2..2+D) of mapped host memory, then the
// completion signal.  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_import_signal(const uint32_t *part, int nblk, uint32_t *err, int D,
                                                       HostSignal sig) {
    __shared__ uint32_t s_red[4][256];
    uint32_t r[4] = {0u, 0u, 0u, 0u};
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int k = 0; k < 4; ++k) r[k] = k == 3 ? (r[k] | part[4 * b + k]) : max(r[k], part[4 * b + k]);
    for (int k = 0; k < 4; ++k) s_red[k][threadIdx.x] = r[k];
    __syncthreads();
    if (threadIdx.x != 0) return;
    uint32_t t[4] = {0u, 0u, 0u, 0u};
    for (int j = 0; j < 256; ++j)
        for (int k = 0; k < 4; ++k) t[k] = k == 3 ? (t[k] | s_red[k][j]) : max(t[k], s_red[k][j]);
    err[0] = t[3] & 1u;
    err[1] = (t[3] >> 1) & 1u;
    for (int a = 0; a < D; ++a) err[2 + a] = t[a];
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
    const unsigned grid = grid_for(std::max(n_vertices * dim, n_faces));
    uint32_t *part = nullptr;   // four words per workgroup
    st = dev_alloc(ctx->mem, &part, (size_t)4 * grid, s);
    if (st != AGAL_OK) {
        agal_destroy_geom(g);
        return st;
    }
    {
        ProfScope prof(ctx, "import", s);
        if (dim == 3)
            hipLaunchKernelGGL(k_import<3>, dim3(grid), dim3(256), 0, s, d_vertices, n_vertices, d_faces, n_faces,
                               g->coords, g->aabb, g->rec, g->fidx, part);
        else
            hipLaunchKernelGGL(k_import<2>, dim3(grid), dim3(256), 0, s, d_vertices, n_vertices, d_faces, n_faces,
                               g->coords, g->aabb, g->rec, g->fidx, part);
        hipLaunchKernelGGL(k_import_signal, dim3(1), dim3(256), 0, s, part, (int)grid, err, dim, sig);
    }
    dev_free(ctx->mem, part, s);
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
