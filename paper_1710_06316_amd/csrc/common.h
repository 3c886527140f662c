// Internal declarations shared by the HIP translation units of libafmpb.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/afmpb.h"

#include <atomic>
#include <mutex>
#include <shared_mutex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

namespace afmpb {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

enum : int {
    ST_INVALID = -1, ST_MESH = -2, ST_OOM = -3, ST_NOT_CONVERGED = -4,
    ST_NUMERIC = -5, ST_DEVICE = -6, ST_STATE = -7
};

#define HIPCHK(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            throw ::afmpb::Error(e_ == hipErrorOutOfMemory ? ::afmpb::ST_OOM      \
                                                           : ::afmpb::ST_DEVICE,  \
                                 std::string(#call) + ": " + hipGetErrorString(e_)); \
        }                                                                         \
    } while (0)

#define KCHK() HIPCHK(hipGetLastError())

inline void require(bool ok, int code, const std::string &msg) {
    if (!ok) throw Error(code, msg);
}

// ---------------------------------------------------------------------------
// Device buffer (owning, move-only)
// ---------------------------------------------------------------------------

// Device bytes held by DBufs are added to the counter that is current on the
// allocating thread (if any) and taken off it again on release; the solve
// server uses this for its memory budget.
inline thread_local std::atomic<long long> *g_dev_bytes = nullptr;

// Device frees (which may synchronise the device) never overlap a graph
// capture in another thread: frees hold this lock shared, captures hold it
// exclusively.
inline std::shared_mutex g_capture_mu;

// The caller-supplied device memory supplier of the context whose entry
// point runs on this thread (null: hipMalloc / hipFree), and that context's
// stream; set for the duration of each context call.
inline thread_local const afmpb_allocator *g_alloc = nullptr;
inline thread_local hipStream_t g_alloc_stream = nullptr;

struct AllocScope {
    const afmpb_allocator *a0;
    hipStream_t s0;
    AllocScope(const afmpb_allocator *a, hipStream_t s) : a0(g_alloc), s0(g_alloc_stream) {
        g_alloc = a;
        g_alloc_stream = s;
    }
    ~AllocScope() {
        g_alloc = a0;
        g_alloc_stream = s0;
    }
};

// Device memory released while a DeferFree scope is open on this thread is
// returned when the scope closes, after a device synchronisation, instead of
// at once: a free waits for the whole device, which would serialise the
// setup with work left running on another stream meanwhile.
struct Deferred {
    void *p;
    const afmpb_allocator *al;
    std::atomic<long long> *acct;
    long long bytes;
};
inline thread_local std::vector<Deferred> *g_defer = nullptr;

inline void free_now(void *p, const afmpb_allocator *al) {
    if (al) {
        // the supplier may hand the memory out again at once: wait for every
        // queued use of it first
        (void)hipDeviceSynchronize();
        al->free(p, al->user);
    } else {
        std::shared_lock<std::shared_mutex> lk(g_capture_mu);
        (void)hipFree(p);
    }
}

struct DeferFree {
    std::vector<Deferred> list;
    std::vector<Deferred> *prev;
    DeferFree() : prev(g_defer) { g_defer = &list; }
    DeferFree(const DeferFree &) = delete;
    DeferFree &operator=(const DeferFree &) = delete;
    ~DeferFree() {
        g_defer = prev;
        if (list.empty()) return;
        (void)hipDeviceSynchronize();
        for (const Deferred &d : list) {
            free_now(d.p, d.al);
            if (d.acct) *d.acct -= d.bytes;
        }
    }
};

template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    std::atomic<long long> *acct = nullptr;
    const afmpb_allocator *al = nullptr;    // supplier of p (null: hipMalloc)
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n), acct(o.acct), al(o.al) {
        o.p = nullptr; o.n = 0; o.acct = nullptr; o.al = nullptr;
    }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; acct = o.acct; al = o.al;
            o.p = nullptr; o.n = 0; o.acct = nullptr; o.al = nullptr;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) count = 1;  // keep a valid pointer for empty arrays
        const size_t bytes = count * sizeof(T);
        if (g_alloc) {
            // 256-byte granules: every buffer starts aligned for wide loads
            void *q = g_alloc->alloc((bytes + 255) / 256 * 256, (void *)g_alloc_stream, g_alloc->user);
            if (!q) throw Error(ST_OOM, "device allocation by the caller's allocator failed");
            p = static_cast<T *>(q);
            al = g_alloc;
        } else {
            HIPCHK(hipMalloc(reinterpret_cast<void **>(&p), bytes));
        }
        n = count;
        acct = g_dev_bytes;
        if (acct) *acct += (long long)(n * sizeof(T));
    }
    void release() {
        if (p) {
            if (g_defer) {
                g_defer->push_back({p, al, acct, (long long)(n * sizeof(T))});
            } else {
                free_now(p, al);
                if (acct) *acct -= (long long)(n * sizeof(T));
            }
            p = nullptr; n = 0; acct = nullptr; al = nullptr;
        }
    }
    T *get() const { return p; }
    void upload(const T *h, size_t count, hipStream_t s) {
        if (count) HIPCHK(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void download(T *h, size_t count, hipStream_t s) const {
        if (count) HIPCHK(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
    void zero(size_t count, hipStream_t s) {
        if (count) HIPCHK(hipMemsetAsync(p, 0, count * sizeof(T), s));
    }
};

// P2P lane replication: a target group of n points runs as f copies of
// 64/f lanes, each copy taking every f-th source (f = 8, 4, 2, 1).
__host__ __device__ inline int p2p_replicas(int ntarget) {
    return ntarget <= 8 ? 8 : ntarget <= 16 ? 4 : ntarget <= 32 ? 2 : 1;
}

// Blocks for n threads.  A dispatch's grid size per dimension is a 32-bit
// count of work-items, so a launch of 2^32 or more threads would silently
// drop work: refuse it (large loops use a capped grid and a stride).
inline unsigned blocks_ok(long long blocks, long long block) {
    require(blocks >= 1 && blocks * block < (1ll << 32), -1, "launch larger than 2^32 work-items");
    return (unsigned)blocks;
}
inline unsigned grid_for(long long n, int block) {
    long long g = (n + block - 1) / block;
    if (g < 1) g = 1;
    require(g * (long long)block < (1ll << 32), -1, "launch larger than 2^32 work-items");
    return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Primitives (prims.hip)
// ---------------------------------------------------------------------------

// Exclusive prefix sum of in[0..n) into out[0..n]; out[n] = total.  in and out
// may alias.  Returns nothing; the caller reads out[n] when it needs the total.
void exclusive_scan_i32(const int *in, int *out, long long n, hipStream_t s);
void exclusive_scan_i64(const long long *in, long long *out, long long n, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys.  Sorted results end in keys/vals (the scratch buffers are used as
// ping-pong storage and must hold n elements each).
void radix_sort_pairs(unsigned long long *keys, int *vals,
                      unsigned long long *tmp_keys, int *tmp_vals, long long n,
                      int bits, hipStream_t s);

// Sort each CSR row ascending (rows are short; one thread per row).
void sort_rows_i32(const int *ptr, int *idx, long long nrows, hipStream_t s);

// ---------------------------------------------------------------------------
// Profiling (api.hip)
// ---------------------------------------------------------------------------

struct Prof;
struct ProfScope {
    Prof *prof; int id; hipStream_t s; size_t slot;
    ProfScope(Prof *p, const char *name, hipStream_t st);
    ~ProfScope();
};

}  // namespace afmpb
