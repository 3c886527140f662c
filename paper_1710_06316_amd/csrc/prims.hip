// Device primitives: exclusive scan, stable LSD radix sort of (key, value)
// pairs, per-row sort of short CSR rows.  Written for 64-lane wavefronts.
#include "common.h"

namespace afmpb {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <typename T>
__device__ T wave_inclusive_scan(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive scan of the block's per-thread values; returns the block total.
template <typename T>
__device__ T block_exclusive_scan(T v, T &excl) {
    __shared__ T wsum[SCAN_BLOCK / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    T before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    excl = before + inc - v;
    __syncthreads();
    return total;
}

template <typename T>
__global__ void k_scan_reduce(const T *in, long long n, T *sums) {
    long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    T s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    T excl;
    T tot = block_exclusive_scan(s, excl);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ void k_scan_apply(const T *in, T *out, long long n, const T *offs, int add_total) {
    long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
    T loc[SCAN_ITEMS];
    T s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        loc[i] = (base + i < n) ? in[base + i] : T(0);
        s += loc[i];
    }
    T excl;
    T tot = block_exclusive_scan(s, excl);
    T off = offs ? offs[blockIdx.x] : T(0);
    T run = off + excl;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += loc[i];
    }
    if (add_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + tot;
}

template <typename T>
void exclusive_scan(const T *in, T *out, long long n, hipStream_t s) {
    if (n <= 0) {
        T z = 0;
        HIPCHK(hipMemcpyAsync(out, &z, sizeof(T), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        return;
    }
    long long nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        k_scan_apply<T><<<1, SCAN_BLOCK, 0, s>>>(in, out, n, nullptr, 1);
        KCHK();
        return;
    }
    DBuf<T> sums(nb + 1);
    k_scan_reduce<T><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, n, sums.p);
    KCHK();
    exclusive_scan<T>(sums.p, sums.p, nb, s);
    k_scan_apply<T><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, out, n, sums.p, 1);
    KCHK();
    HIPCHK(hipStreamSynchronize(s));  // sums is freed on return
}

// ----------------------------- radix sort ----------------------------------

constexpr int RS_BLOCK = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;
constexpr int RS_WAVES = RS_BLOCK / 64;

__global__ void k_rs_hist(const unsigned long long *keys, long long n, int shift,
                          int *hist, int nblk) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    long long base = (long long)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_ITEMS; ++i) {
        long long idx = base + (long long)i * RS_BLOCK + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(long long)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: items are visited in index order (iteration-major, then
// thread); equal digits keep their order via wave ballots plus per-wave
// digit counts.
__global__ void k_rs_scatter(const unsigned long long *kin, const int *vin,
                             unsigned long long *kout, int *vout, long long n,
                             int shift, const int *offs, int nblk, int *err) {
    __shared__ int run[256];
    __shared__ int wcnt[RS_WAVES][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    run[tid] = offs[(long long)tid * nblk + blockIdx.x];
    for (int w = 0; w < RS_WAVES; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    long long base = (long long)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_ITEMS; ++i) {
        long long idx = base + (long long)i * RS_BLOCK + tid;
        bool valid = idx < n;
        unsigned long long k = valid ? kin[idx] : 0ull;
        int v = valid ? vin[idx] : 0;
        int d = (int)((k >> shift) & 255u);
        unsigned long long mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1;
            unsigned long long bb = __ballot(valid && bit);
            mask &= bit ? bb : ~bb;
        }
        int rank = __popcll(mask & lt);
        int cnt = __popcll(mask);
        if (valid && rank == cnt - 1) wcnt[wave][d] = cnt;
        __syncthreads();
        if (valid) {
            int pre = 0;
            for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
            int pos = run[d] + pre + rank;
            if (pos < 0 || pos >= n) {
                atomicOr(err, 1);
            } else {
                kout[pos] = k;
                vout[pos] = v;
            }
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < RS_WAVES; ++w) { add += wcnt[w][tid]; wcnt[w][tid] = 0; }
        run[tid] += add;
        __syncthreads();
    }
}

__global__ void k_sort_rows(const int *ptr, int *idx, long long nrows) {
    long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    int b = ptr[r], e = ptr[r + 1];
    for (int i = b + 1; i < e; ++i) {
        int v = idx[i];
        int j = i - 1;
        while (j >= b && idx[j] > v) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
}

}  // namespace

void exclusive_scan_i32(const int *in, int *out, long long n, hipStream_t s) {
    exclusive_scan<int>(in, out, n, s);
}
void exclusive_scan_i64(const long long *in, long long *out, long long n, hipStream_t s) {
    exclusive_scan<long long>(in, out, n, s);
}

void radix_sort_pairs(unsigned long long *keys, int *vals, unsigned long long *tk,
                      int *tv, long long n, int bits, hipStream_t s) {
    if (n <= 1) return;
    require(n < (1ll << 31), ST_INVALID, "radix sort: too many elements");
    int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
    DBuf<int> hist((size_t)256 * nblk + 1), err(1);
    err.zero(1, s);
    int passes = (bits + 7) / 8;
    unsigned long long *ka = keys, *kb = tk;
    int *va = vals, *vb = tv;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        k_rs_hist<<<nblk, RS_BLOCK, 0, s>>>(ka, n, shift, hist.p, nblk);
        KCHK();
        exclusive_scan_i32(hist.p, hist.p, (long long)256 * nblk, s);
        k_rs_scatter<<<nblk, RS_BLOCK, 0, s>>>(ka, va, kb, vb, n, shift, hist.p, nblk, err.p);
        KCHK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        HIPCHK(hipMemcpyAsync(keys, ka, n * sizeof(unsigned long long), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(vals, va, n * sizeof(int), hipMemcpyDeviceToDevice, s));
    }
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));  // hist is freed on return
    require(herr == 0, ST_DEVICE, "radix sort: scatter index out of range");
}

void sort_rows_i32(const int *ptr, int *idx, long long nrows, hipStream_t s) {
    if (nrows <= 0) return;
    k_sort_rows<<<grid_for(nrows, 256), 256, 0, s>>>(ptr, idx, nrows);
    KCHK();
}

}  // namespace afmpb
