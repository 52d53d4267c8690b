// Runtime pieces of the library: error reporting, the device allocator,
// fill kernels, the single-pass exclusive scan and small read-backs.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>

#include "agal_internal.hpp"
#include "device.hpp"

namespace agal {

static thread_local char g_err[512] = "";

agal_status fail(agal_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

uint64_t next_handle_id() {
    static std::atomic<uint64_t> next{1};
    return next.fetch_add(1);
}

// 256-byte granules up to 4 KiB, then eight classes per octave (at most 12.5 %
// slack).
size_t Allocator::size_class(size_t bytes) {
    if (bytes <= 4096) return (bytes + 255) & ~size_t(255);
    int e = 63 - __builtin_clzll((unsigned long long)bytes);
    const size_t step = size_t(1) << (e - 3);
    return (bytes + step - 1) & ~(step - 1);
}

void *Allocator::alloc(size_t bytes, hipStream_t s) const {
    if (has_user) return user.alloc(user.ctx, bytes, (void *)s);
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto range = cached.equal_range(cls);
        for (auto it = range.first; it != range.second; ++it)
            if (it->second.s == s) {
                void *p = it->second.p;
                cached.erase(it);
                cached_bytes -= cls;
                live[p] = cls;
                return p;
            }
    }
    void *p = nullptr;
    if (hipMallocAsync(&p, cls, s) != hipSuccess) {
        (void)hipGetLastError();
        drain();   // give cached blocks back to the pool and try once more
        if (hipMallocAsync(&p, cls, s) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lk(mu);
    live[p] = cls;
    return p;
}

void Allocator::release(void *p, hipStream_t s) const {
    if (!p) return;
    if (has_user) {
        user.free(user.ctx, p, (void *)s);
        return;
    }
    std::lock_guard<std::mutex> lk(mu);
    auto it = live.find(p);
    if (it == live.end()) {
        (void)hipFreeAsync(p, s);
        return;
    }
    const size_t cls = it->second;
    live.erase(it);
    if (cached_bytes + cls > kCacheCap) {
        (void)hipFreeAsync(p, s);
        return;
    }
    cached.emplace(cls, Block{p, s});
    cached_bytes += cls;
}

void Allocator::drain() const {
    if (has_user) return;
    std::lock_guard<std::mutex> lk(mu);
    if (cached.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : cached) (void)hipFree(kv.second.p);
    (void)hipGetLastError();
    cached.clear();
    cached_bytes = 0;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
static hipEvent_t take_event(agal_context ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

ProfScope::ProfScope(agal_context ctx, const char *name, hipStream_t s) : ctx_(ctx), name_(name), s_(s) {
    if (!ctx_ || !ctx_->profiling) return;
    start_ = take_event(ctx_);
    if (start_ && hipEventRecord(start_, s_) != hipSuccess) {
        (void)hipGetLastError();
        ctx_->event_pool.push_back(start_);
        start_ = nullptr;
    }
}

ProfScope::~ProfScope() {
    if (!start_) return;
    hipEvent_t stop = take_event(ctx_);
    if (stop && hipEventRecord(stop, s_) == hipSuccess) {
        ctx_->records.push_back({name_, start_, stop});
        return;
    }
    (void)hipGetLastError();
    ctx_->event_pool.push_back(start_);
    if (stop) ctx_->event_pool.push_back(stop);
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
static void fill(T *p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) { fill(p, v, n, s); }
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) { fill(p, v, n, s); }
void fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) { fill(p, v, n, s); }

// ---------------------------------------------------------------------------
// exclusive scan (decoupled look-back)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

struct LoadU32 {
    const uint32_t *p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct LoadFlagU8 {
    const uint8_t *p;
    __device__ uint32_t operator()(int64_t i) const { return p[i] != 0 ? 1u : 0u; }
};
struct LoadPopc64 {
    const unsigned long long *p;
    __device__ uint32_t operator()(int64_t i) const { return (uint32_t)__popcll(p[i]); }
};

HostSignal host_signal(agal_context ctx) {
    return HostSignal{ctx->d_done, ctx->d_counts + kSyncWord, ++ctx->sync_seq};
}

agal_status wait_signal(agal_context ctx, hipStream_t s, const HostSignal &sig, const char *what) {
    // The stream's status is polled only once the wait has lasted a while: a
    // query per few microseconds delays the wake-up by about as much (measured:
    // 0.41 -> 0.47 ms on a six-wait step).
    volatile uint32_t *w = ctx->h_counts + kSyncWord;
    const auto t0 = std::chrono::steady_clock::now();
    bool poll = false;
    for (uint64_t i = 0;; ++i) {
        if (*w == sig.seq) break;
        if ((i & 1023u) == 1023u && !poll) poll = std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(1);
        if (poll && (i & 1023u) == 1023u) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return fail(AGAL_EHIP, "%s: %s", what, hipGetErrorString(e));
            if (*w == sig.seq) break;
            return fail(AGAL_EHIP, "%s: the stream finished without the kernel's completion signal", what);
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return AGAL_OK;
}

template <class In>
__global__ __launch_bounds__(kScanThreads) void k_scan(In in, uint32_t *out, int64_t n, uint64_t *status,
                                                       uint32_t *ticket, uint32_t *host_total, HostSignal sig) {
    __shared__ uint32_t s_tile, s_prefix;
    __shared__ uint32_t s_wsum[kScanThreads / dev::kWave];
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? in(idx) : 0u;
        sum += v[i];
    }
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x % dev::kWave;
    uint32_t incl = dev::wave_inclusive_sum(sum);
    if (lane == dev::kWave - 1) s_wsum[w] = incl;
    __syncthreads();
    uint32_t wpre = 0, total = 0;
#pragma unroll
    for (int j = 0; j < kScanThreads / dev::kWave; ++j) {
        if (j < w) wpre += s_wsum[j];
        total += s_wsum[j];
    }
    if (w == 0) {
        uint32_t p = dev::lookback_wave(status, tile, total);
        if (lane == 0) s_prefix = p;
    }
    __syncthreads();
    uint32_t run = s_prefix + wpre + incl - sum;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
        if (idx == n - 1) {
            out[n] = run;
            // the total is known once this tile's look-back ends: the host
            // needs nothing else from this launch
            if (host_total) {
                *host_total = run;
                dev::publish_host(sig.word, sig.seq);
            }
        }
    }
}

agal_status lookback_alloc(agal_context ctx, int64_t tiles, uint64_t **status, uint32_t **ticket, hipStream_t s) {
    // one buffer: status words then the ticket
    uint64_t *buf = nullptr;
    AGAL_TRY(dev_alloc(ctx->mem, &buf, (size_t)tiles + 1, s));
    fill_u64(buf, 0ull, tiles + 1, s);
    *status = buf;
    *ticket = reinterpret_cast<uint32_t *>(buf + tiles);
    return AGAL_OK;
}

// status: tiles + 1 zeroed words (look-back status, then the ticket), or null
// to have one allocated and zeroed here.  total: when non-null, the sum is
// written to mapped host memory by the kernel and returned after a stream
// synchronisation (no separate read-back).
template <class In>
static agal_status scan_impl(agal_context ctx, In in, uint32_t *out, int64_t n, hipStream_t s,
                             uint64_t *status = nullptr, uint32_t *total = nullptr, bool timed = true) {
    if (n <= 0) {
        fill_u32(out, 0u, 1, s);
        if (total) *total = 0;
        return AGAL_OK;
    }
    const int64_t tiles = scan_tiles(n);
    const bool own = status == nullptr;
    uint32_t *ticket = nullptr;
    if (own) AGAL_TRY(lookback_alloc(ctx, tiles, &status, &ticket, s));
    else ticket = reinterpret_cast<uint32_t *>(status + tiles);
    const HostSignal sig = total ? host_signal(ctx) : HostSignal{nullptr, nullptr, 0u};
    {
        ProfScope prof(timed ? ctx : nullptr, "scan_exclusive", s);
        hipLaunchKernelGGL(k_scan<In>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n, status, ticket,
                           total ? ctx->d_counts : nullptr, sig);
    }
    if (own) dev_free(ctx->mem, status, s);
    AGAL_TRY_HIP(hipGetLastError());
    if (total) {
        AGAL_TRY(wait_signal(ctx, s, sig, "device scan"));
        *total = ctx->h_counts[0];
    }
    return AGAL_OK;
}

int64_t scan_tiles(int64_t n) { return n <= 0 ? 0 : (n + kScanTile - 1) / kScanTile; }

agal_status scan_u32(agal_context ctx, const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s) {
    return scan_impl(ctx, LoadU32{in}, out, n, s);
}
agal_status scan_u32_total(agal_context ctx, const uint32_t *in, uint32_t *out, int64_t n, uint64_t *status,
                           uint32_t *total, hipStream_t s, bool timed) {
    return scan_impl(ctx, LoadU32{in}, out, n, s, status, total, timed);
}
agal_status scan_popc64_total(agal_context ctx, const unsigned long long *masks, uint32_t *out, int64_t n,
                              uint32_t *total, hipStream_t s) {
    return scan_impl(ctx, LoadPopc64{masks}, out, n, s, nullptr, total);
}
agal_status scan_flags_u8(agal_context ctx, const uint8_t *in, uint32_t *out, int64_t n, hipStream_t s) {
    return scan_impl(ctx, LoadFlagU8{in}, out, n, s);
}

// Several flag scans in one launch: the tiles of all arrays share one ticket
// counter, so every array's tiles are taken in order and each looks back only
// over its own array's status words.
__global__ __launch_bounds__(kScanThreads) void k_scan_flags_multi(MultiScanArgs a, uint64_t *status,
                                                                    uint32_t *ticket) {
    __shared__ uint32_t s_tile, s_prefix;
    __shared__ uint32_t s_wsum[kScanThreads / dev::kWave];
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t gtile = s_tile;
    int seg = 0;
    while (seg + 1 < a.nseg && a.tile0[seg + 1] <= gtile) ++seg;
    const uint32_t tile = gtile - a.tile0[seg];
    const uint8_t *in = a.in[seg];
    uint32_t *out = a.out[seg];
    const int64_t n = a.n[seg];
    const int64_t base = (int64_t)tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < n ? (in[idx] != 0 ? 1u : 0u) : 0u;
        sum += v[i];
    }
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x % dev::kWave;
    const uint32_t incl = dev::wave_inclusive_sum(sum);
    if (lane == dev::kWave - 1) s_wsum[w] = incl;
    __syncthreads();
    uint32_t wpre = 0, total = 0;
#pragma unroll
    for (int j = 0; j < kScanThreads / dev::kWave; ++j) {
        if (j < w) wpre += s_wsum[j];
        total += s_wsum[j];
    }
    if (w == 0) {
        const uint32_t p = dev::lookback_wave(status + a.tile0[seg], tile, total);
        if (lane == 0) s_prefix = p;
    }
    __syncthreads();
    uint32_t run = s_prefix + wpre + incl - sum;
    // the thread holding an array's last element (tile 0's first thread for
    // an empty array) reports its total, and the last of the k reports adds
    // the extra word and signals the host
    bool report = false;
    if (n == 0 && threadIdx.x == 0) {
        out[0] = 0u;
        a.host_total[seg] = 0u;
        report = true;
    }
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
        if (idx == n - 1) {
            out[n] = run;
            a.host_total[seg] = run;
            report = true;
        }
    }
    if (report && dev::arrive_last(a.sig.done, (uint32_t)a.nseg)) {
        a.host_total[a.nseg] = a.extra ? *a.extra : 0u;
        dev::publish_host(a.sig.word, a.sig.seq);
    }
}

int64_t scan_flags_u8_multi_tiles(const int64_t *n, int k) {
    int64_t tiles = 0;
    for (int i = 0; i < k; ++i) tiles += std::max<int64_t>(1, (n[i] + kScanTile - 1) / kScanTile);
    return tiles;
}

agal_status scan_flags_u8_multi(agal_context ctx, const uint8_t *const *in, uint32_t *const *out, const int64_t *n,
                                int k, const uint32_t *extra, uint32_t *totals, hipStream_t s, uint64_t *status_zeroed) {
    if (k <= 0) return AGAL_OK;
    if (k > kMultiScanMax) return fail(AGAL_EINVAL, "scan_flags_u8_multi: at most %d arrays", kMultiScanMax);
    MultiScanArgs a{};
    a.nseg = k;
    a.extra = extra;
    a.host_total = ctx->d_counts;
    a.sig = host_signal(ctx);
    uint32_t tiles = 0;
    for (int i = 0; i < k; ++i) {
        a.in[i] = in[i];
        a.out[i] = out[i];
        a.n[i] = n[i];
        a.tile0[i] = tiles;
        tiles += (uint32_t)std::max<int64_t>(1, (n[i] + kScanTile - 1) / kScanTile);   // an empty array still writes out[0]
    }
    uint64_t *status = status_zeroed;
    uint32_t *ticket = nullptr;
    if (status) ticket = reinterpret_cast<uint32_t *>(status + tiles);
    else AGAL_TRY(lookback_alloc(ctx, tiles, &status, &ticket, s));
    {
        ProfScope prof(ctx, "scan_exclusive", s);
        hipLaunchKernelGGL(k_scan_flags_multi, dim3(tiles), dim3(kScanThreads), 0, s, a, status, ticket);
    }
    if (!status_zeroed) dev_free(ctx->mem, status, s);
    AGAL_TRY_HIP(hipGetLastError());
    AGAL_TRY(wait_signal(ctx, s, a.sig, "mark scan"));
    for (int i = 0; i <= k; ++i) totals[i] = ctx->h_counts[i];
    return AGAL_OK;
}


// ---------------------------------------------------------------------------
// lattices
// ---------------------------------------------------------------------------
bool lattice_table(int Q, Lattice *out) {
    Lattice L;
    L.Q = Q;
    if (Q == AGAL_D2Q9) L.dim = 2;
    else if (Q == AGAL_D3Q19 || Q == AGAL_D3Q27) L.dim = 3;
    else return false;
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < 3; ++a) L.c[i][a] = L.dim == 3 ? kDir3[i][a] : kDir2[i][a];
    *out = L;
    return true;
}

}  // namespace agal

// ---------------------------------------------------------------------------
// C ABI: context, status strings, lattice vectors
// ---------------------------------------------------------------------------
extern "C" {

agal_status agal_context_create(const agal_allocator *alloc, agal_context *out) {
    if (!out) return agal::fail(AGAL_EINVAL, "agal_context_create: out is NULL");
    if (alloc && (!alloc->alloc || !alloc->free))
        return agal::fail(AGAL_EINVAL, "agal_context_create: allocator needs alloc and free");
    int dev = 0;
    AGAL_TRY_HIP(hipGetDevice(&dev));
    auto *c = new (std::nothrow) agal_context_t();
    if (!c) return agal::fail(AGAL_ENOMEM, "agal_context_create: host allocation failed");
    c->device = dev;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        c->n_cu = ncu;
    (void)hipGetLastError();
    if (alloc) {
        c->mem.user = *alloc;
        c->mem.has_user = true;
    } else {
        // keep freed blocks in the stream-ordered pool instead of returning them to the driver
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        (void)hipGetLastError();
    }
    c->h_counts_cap = 64;
    if (hipHostMalloc((void **)&c->h_counts, c->h_counts_cap * sizeof(uint32_t),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->d_counts, c->h_counts, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (c->h_counts) (void)hipHostFree(c->h_counts);
        delete c;
        return agal::fail(AGAL_ENOMEM, "agal_context_create: mapped pinned host allocation failed");
    }
    c->h_counts[agal::kSyncWord] = 0u;
    if (hipMalloc((void **)&c->d_done, 8 * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->d_done, 0, 8 * sizeof(uint32_t)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        if (c->d_done) (void)hipFree(c->d_done);
        (void)hipHostFree(c->h_counts);
        delete c;
        return agal::fail(AGAL_ENOMEM, "agal_context_create: device counter allocation failed");
    }
    // the device address of the binning scratch array, taken once per device
    // (a failure here only disables agal_bin_faces_noalloc, which reports it)
    (void)agal::bin_scratch_resolve(dev);
    *out = c;
    return AGAL_OK;
}

void agal_context_destroy(agal_context ctx) {
    if (!ctx) return;
    ctx->mem.drain();
    for (auto &r : ctx->records) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->h_counts) (void)hipHostFree(ctx->h_counts);
    if (ctx->d_done) (void)hipFree(ctx->d_done);
    delete ctx;
}

agal_status agal_context_set_flag_table_limit(agal_context ctx, int64_t max_entries) {
    if (!ctx) return agal::fail(AGAL_EINVAL, "agal_context_set_flag_table_limit: NULL context");
    if (max_entries < 0) return agal::fail(AGAL_EINVAL, "agal_context_set_flag_table_limit: negative limit");
    ctx->flag_table_max = max_entries;
    return AGAL_OK;
}

agal_status agal_context_set_link_list_limit(agal_context ctx, int64_t max_blocks_per_face) {
    if (!ctx) return agal::fail(AGAL_EINVAL, "agal_context_set_link_list_limit: NULL context");
    if (max_blocks_per_face < 0)
        return agal::fail(AGAL_EINVAL, "agal_context_set_link_list_limit: negative limit");
    ctx->link_list_max = max_blocks_per_face;
    return AGAL_OK;
}

agal_status agal_profile_enable(agal_context ctx, int enable) {
    if (!ctx) return agal::fail(AGAL_EINVAL, "agal_profile_enable: NULL context");
    ctx->profiling = enable != 0;
    return AGAL_OK;
}

agal_status agal_profile_read(agal_context ctx, int max_entries, const char **names, int64_t *launches,
                              double *total_ms, int *n_entries) {
    if (!ctx || !n_entries) return agal::fail(AGAL_EINVAL, "agal_profile_read: NULL argument");
    if (max_entries > 0 && (!names || !launches || !total_ms))
        return agal::fail(AGAL_EINVAL, "agal_profile_read: NULL output array");
    int n = 0;
    for (auto &r : ctx->records) {
        AGAL_TRY_HIP(hipEventSynchronize(r.stop));
        float ms = 0.0f;
        AGAL_TRY_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
        int k = 0;
        while (k < n && strcmp(names[k], r.name) != 0) ++k;
        if (k == n) {
            if (n == max_entries) continue;
            names[n] = r.name;
            launches[n] = 0;
            total_ms[n] = 0.0;
            ++n;
        }
        launches[k] += 1;
        total_ms[k] += ms;
    }
    for (auto &r : ctx->records) {
        ctx->event_pool.push_back(r.start);
        ctx->event_pool.push_back(r.stop);
    }
    ctx->records.clear();
    *n_entries = n;
    return AGAL_OK;
}

const char *agal_status_string(agal_status s) {
    switch (s) {
        case AGAL_OK: return "AGAL_OK";
        case AGAL_EINVAL: return "AGAL_EINVAL: invalid argument";
        case AGAL_ENOMEM: return "AGAL_ENOMEM: out of memory";
        case AGAL_EHIP: return "AGAL_EHIP: HIP runtime error";
        case AGAL_ECAPACITY: return "AGAL_ECAPACITY: capacity exceeded";
        case AGAL_ESTATE: return "AGAL_ESTATE: inconsistent handles or state";
    }
    return "unknown agal_status";
}

const char *agal_last_error(void) { return agal::g_err; }

agal_status agal_lattice_vectors(int lattice, int32_t *c) {
    agal::Lattice L;
    if (!agal::lattice_table(lattice, &L)) return agal::fail(AGAL_EINVAL, "unknown lattice %d", lattice);
    if (!c) return agal::fail(AGAL_EINVAL, "agal_lattice_vectors: c is NULL");
    for (int i = 0; i < lattice; ++i)
        for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    return AGAL_OK;
}

}  // extern "C"
