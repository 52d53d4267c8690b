// Private declarations of the HIP library: handle layouts, allocation and
// error plumbing, and the launchers each translation unit exports to the
// others.  Device arithmetic lives in device.hpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "agal.h"

namespace agal {

constexpr int kMaxLevels = AGAL_MAX_LEVELS;

// Records a message for agal_last_error() and returns `s`.
agal_status fail(agal_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define AGAL_TRY_HIP(expr)                                                                   \
    do {                                                                                     \
        hipError_t e__ = (expr);                                                             \
        if (e__ != hipSuccess)                                                               \
            return ::agal::fail(AGAL_EHIP, "%s failed: %s", #expr, hipGetErrorString(e__));  \
    } while (0)

#define AGAL_TRY(expr)                              \
    do {                                            \
        agal_status s__ = (expr);                   \
        if (s__ != AGAL_OK) return s__;             \
    } while (0)

// Device memory through the context's allocator: the user's callbacks, or a
// caching layer over the HIP stream-ordered pool.  Every allocation is stream
// ordered.  The cache keeps released blocks by size class and hands a block
// out again only to an allocation on the stream it was released on (work on
// one stream runs in order, so no event is needed); blocks beyond kCacheCap
// bytes go back to the pool.
struct Allocator {
    agal_allocator user{};
    bool has_user = false;
    static constexpr size_t kCacheCap = size_t(16) << 30;
    struct Block {
        void *p;
        hipStream_t s;
    };
    mutable std::mutex mu;
    mutable std::multimap<size_t, Block> cached;                    // size class -> released block
    mutable std::unordered_map<void *, size_t> live;                // block -> its size class
    mutable size_t cached_bytes = 0;
    static size_t size_class(size_t bytes);
    void *alloc(size_t bytes, hipStream_t s) const;
    void release(void *p, hipStream_t s) const;
    void drain() const;   // returns every cached block (device synchronised first)
};

template <class T>
inline agal_status dev_alloc(const Allocator &a, T **p, size_t count, hipStream_t s) {
    *p = nullptr;
    if (count == 0) count = 1;
    void *q = a.alloc(count * sizeof(T), s);
    if (!q) return fail(AGAL_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
    *p = static_cast<T *>(q);
    return AGAL_OK;
}

template <class T>
inline void dev_free(const Allocator &a, T *&p, hipStream_t s) {
    if (p) a.release(p, s);
    p = nullptr;
}

uint64_t next_handle_id();

}  // namespace agal

namespace agal {
struct ProfRecord {
    const char *name;
    hipEvent_t start, stop;
};
}  // namespace agal

struct agal_context_t {
    agal::Allocator mem;
    int device = 0;
    int n_cu = 256;                 // compute units of the device
    // small pinned host buffer for count read-backs
    uint32_t *h_counts = nullptr;   // mapped pinned host memory
    uint32_t *d_counts = nullptr;   // its device address
    size_t h_counts_cap = 0;
    // kernel timing (HIP events around each launch) when enabled
    bool profiling = false;
    int64_t flag_table_max = int64_t(1) << 24;   // agal_context_set_flag_table_limit
    int64_t link_list_max = 512;                  // agal_context_set_link_list_limit
    // completion signals: a device arrival counter d_done[0] (zero between
    // kernels) and the sequence number last handed out; the signal word is
    // h_counts[kSyncWord]
    uint32_t *d_done = nullptr;
    uint32_t sync_seq = 0;
    std::vector<agal::ProfRecord> records;
    std::vector<hipEvent_t> event_pool;
};

struct agal_geom_t {
    agal_context ctx = nullptr;
    uint64_t id = 0;
    hipStream_t stream = nullptr;
    int dim = 0;
    int64_t F = 0, Nv = 0;
    float *coords = nullptr;   // (dim*dim) x F
    float *aabb = nullptr;     // (2*dim) x F
    float *rec = nullptr;      // F x (16 in 3D, 8 in 2D): corners, min, max
    int32_t *fidx = nullptr;   // F x dim
    float max_extent[3] = {};  // largest face bounding-box extent per axis
};

struct agal_bins_t {
    agal_context ctx = nullptr;
    uint64_t geom_id = 0;
    hipStream_t stream = nullptr;
    int dim = 0, B = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, s[3] = {0, 0, 0};
    int64_t nb = 0, P = 0;
    uint32_t *off = nullptr;   // nb + 1
    int32_t *ids = nullptr;    // P
    bool discrete = false;     // faces binned by their sampled points (not a superset of the box bins)
    float spacing = 0.0f;      // sample spacing of the discrete binning
};

namespace agal {
struct Level {
    int64_t n = 0;
    uint32_t *keys = nullptr;
    uint8_t *leaf = nullptr;
    uint8_t *mark = nullptr;   // export mark: 1 flagged, 2 balance
    uint8_t *cf = nullptr;     // per-cell flags (levels that were tested)
};
}  // namespace agal

struct agal_forest_t {
    agal_context ctx = nullptr;
    uint64_t geom_id = 0;
    hipStream_t stream = nullptr;
    int dim = 0, L = 0;
    int roots[3] = {1, 1, 1};
    float lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
    float dx[agal::kMaxLevels + 1][3] = {};
    float d[agal::kMaxLevels] = {};
    agal::Level lev[agal::kMaxLevels + 1];
};

struct agal_links_t {
    agal_context ctx = nullptr;
    uint64_t geom_id = 0;
    hipStream_t stream = nullptr;
    int dim = 0, Q = 0, L = 0;
    int roots[3] = {1, 1, 1};
    float lo[3] = {0, 0, 0};
    float dx[3] = {0, 0, 0};
    int64_t n = 0;
    uint64_t *key = nullptr;
    float *q = nullptr;
    int32_t *face = nullptr;
};

namespace agal {

// Lattice table shared by the link and adjoint kernels (host copy; kernels
// receive it by value).
struct Lattice {
    int Q = 0;
    int dim = 0;
    int8_t c[27][3] = {};
};
bool lattice_table(int Q, Lattice *out);

// Device-wide exclusive scan of `n` 0/1-or-count values into out[0..n]
// (out[n] = total).  The input is either uint32 counts or uint8 flags
// (nonzero = 1).  Scratch is allocated from the context.
agal_status scan_u32(agal_context ctx, const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s);
agal_status scan_flags_u8(agal_context ctx, const uint8_t *in, uint32_t *out, int64_t n, hipStream_t s);
// k exclusive scans of 0/1 flags (out[i] of length n[i] + 1) in one launch; k <= kMultiScanMax.
constexpr int kMultiScanMax = kMaxLevels + 1;
// Candidate cells of the largest face in a face-centric flag step: per axis its
// box extent plus h + eps on both sides, in cells, plus two for rounding.  A
// level takes the face-centric step only while this stays within
// kFaceFlagMaxPairs: one wave takes 16 faces, so a face far larger than the
// cells would make its wave the whole pass.
constexpr double kFaceFlagMaxPairs = 4096.0;
inline double face_flag_pairs(int D, const float ext[3], float h, const float dx[3], const float eps[3]) {
    double p = 1.0;
    for (int a = 0; a < D; ++a)
        p *= std::floor(((double)ext[a] + 2.0 * ((double)h + (double)eps[a])) / (double)dx[a]) + 2.0;
    return p;
}

// A kernel's completion signal (see dev::publish_host, dev::arrive_last): arrival counter, the
// device address of the mapped signal word (null: none) and the value stored.
struct HostSignal {
    uint32_t *done;
    uint32_t *word;
    uint32_t seq;
};
constexpr int kSyncWord = 63;   // index in the context's mapped words
HostSignal host_signal(agal_context ctx);
// Waits until the kernel that carries `sig` has signalled (spinning on the
// mapped word, with the stream's status checked every so often), in place of
// a stream synchronisation: the host learns of the totals a few microseconds
// after they are written instead of after a runtime wake-up.
agal_status wait_signal(agal_context ctx, hipStream_t s, const HostSignal &sig, const char *what);
struct MultiScanArgs {
    const uint8_t *in[kMultiScanMax];
    uint32_t *out[kMultiScanMax];
    int64_t n[kMultiScanMax];
    uint32_t tile0[kMultiScanMax];
    int nseg;
    const uint32_t *extra;   // one more device word to report (or null: 0)
    uint32_t *host_total;    // mapped host memory: k totals, then *extra
    HostSignal sig;
};
// totals[0..k-1] = sum of each array, totals[k] = *extra; synchronises the stream.  status_zeroed: null, or
// scan_flags_u8_multi_tiles(n, k) + 1 zeroed 64-bit words the caller provides.
agal_status scan_flags_u8_multi(agal_context ctx, const uint8_t *const *in, uint32_t *const *out, const int64_t *n,
                                int k, const uint32_t *extra, uint32_t *totals, hipStream_t s,
                                uint64_t *status_zeroed = nullptr);
int64_t scan_flags_u8_multi_tiles(const int64_t *n, int k);
// Tiles of a scan of n elements; a caller-provided status buffer holds tiles + 1 zeroed 64-bit words.
int64_t scan_tiles(int64_t n);
// Exclusive scan whose sum comes back through mapped host memory (synchronises the stream); status is a
// zeroed buffer of scan_tiles(n) + 1 words, or null.  timed = false: no kernel timing events even when the
// context records them (the no-allocation calls create no events).
agal_status scan_u32_total(agal_context ctx, const uint32_t *in, uint32_t *out, int64_t n, uint64_t *status,
                           uint32_t *total, hipStream_t s, bool timed = true);
// Exclusive scan of the set-bit counts of n 64-bit masks, with the total (synchronises the stream).
agal_status scan_popc64_total(agal_context ctx, const unsigned long long *masks, uint32_t *out, int64_t n,
                              uint32_t *total, hipStream_t s);
// Takes the device address of the binning scratch array for `device` (the
// current device) once; later calls return at once.  Called by
// agal_context_create.
agal_status bin_scratch_resolve(int device);

// Candidate blocks per face along each axis at most, from the largest face box
// extent (bound of the list length); +2 covers the FP64 rounding of the range.
inline double link_blocks_per_face(int D, const float ext[3], const float dx[3], const float eps[3]) {
    double p = 1.0;
    for (int a = 0; a < D; ++a)
        p *= std::floor(((double)ext[a] * (1.0 + 1e-6) + 5.0 * dx[a] + 4.0 * (double)eps[a]) / (4.0 * dx[a])) + 2.0;
    return p;
}

// Link step of one body as agal_link_fractions would take it (used to size
// the batched form): list mode or not, the candidate blocks per face at most,
// and the exact number of candidate-list entries (synchronises s).
struct LinkListPlan {
    bool lists = false;
    int64_t per_face = 0;
    int64_t entries = 0;
};
agal_status link_list_plan(agal_geom g, agal_forest fo, hipStream_t s, LinkListPlan *out);

// Look-back scratch: status words + ticket for `tiles` tiles, cleared.
agal_status lookback_alloc(agal_context ctx, int64_t tiles, uint64_t **status, uint32_t **ticket, hipStream_t s);

// Fill kernels (used instead of hipMemsetAsync so the calls stay capturable).
void fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);

// Records HIP events around the launches in its scope when the context's
// profiling is on; results are aggregated by agal_profile_read.
class ProfScope {
  public:
    ProfScope(agal_context ctx, const char *name, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    agal_context ctx_;
    const char *name_;
    hipStream_t s_;
    hipEvent_t start_ = nullptr;
};


}  // namespace agal
