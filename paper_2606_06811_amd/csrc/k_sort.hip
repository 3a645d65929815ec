// k_sort.hip -- the sorts and scans of the position table (the paper's
// position table of Sec. 5: seed keys grouped with their target positions in
// position order) and of the HSP walking order: a stable least-significant-
// digit radix sort of (key, value) pairs with 8-bit digits, and an exclusive
// prefix sum, both with 64-bit counts.
//
// One radix pass over a digit:
//  1. k_radix_hist: each block counts the digits of its tile of TILE keys;
//     counts go to hist[digit * nblocks + block] (digit-major);
//  2. an exclusive scan of hist turns the counts into each (digit, block)'s
//     first output slot;
//  3. k_radix_scatter: each block walks its tile again in rounds of 256 keys
//     (thread t takes key t of the round, so round-then-thread order is input
//     order) and ranks every key among the keys of the round with the same
//     digit: lanes of one wave with the same digit find each other with eight
//     ballots, waves add up through LDS.  A key goes to its (digit, block)
//     slot plus the keys of its digit in earlier rounds, earlier waves and
//     lower lanes -- so equal digits keep their input order.
#include "sfe_kernels.h"

namespace sfe {

#define SORT_T 256
#define SORT_ROUNDS 16
#define SORT_TILE (SORT_T * SORT_ROUNDS)

template <typename K>
__global__ void __launch_bounds__(SORT_T) k_radix_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                       uint64_t *__restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ROUNDS; r++) {
        const int64_t x = t0 + (int64_t)r * SORT_T + threadIdx.x;
        if (x < n) atomicAdd(&cnt[(uint32_t)(keys[x] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

template <typename K>
__global__ void __launch_bounds__(SORT_T) k_radix_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                          int64_t n, int shift, const uint64_t *__restrict__ slot,
                                                          int64_t nblocks, K *__restrict__ kout,
                                                          uint32_t *__restrict__ vout) {
    __shared__ uint64_t next[256];            // next free output slot per digit for this block
    __shared__ uint32_t wcnt[SORT_T / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    next[tid] = slot[(int64_t)tid * nblocks + blockIdx.x];
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t t0 = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ROUNDS; r++) {
        if (t0 + (int64_t)r * SORT_T >= n) break;             // uniform over the block
#pragma unroll
        for (int q = 0; q < SORT_T / 64; q++) wcnt[q][tid] = 0;
        __syncthreads();
        const int64_t x = t0 + (int64_t)r * SORT_T + tid;
        const bool valid = x < n;
        K key = 0;
        uint32_t val = 0;
        if (valid) { key = kin[x]; val = vin[x]; }
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const uint64_t on = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? on : ~on;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint64_t pos = next[d] + rank;
            for (int q = 0; q < w; q++) pos += wcnt[q][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        {
            uint32_t tot = 0;
#pragma unroll
            for (int q = 0; q < SORT_T / 64; q++) tot += wcnt[q][tid];
            next[tid] += tot;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum: block sums, a scan of the block sums (recursively),
// then each block scans its part from its block's offset.
// ---------------------------------------------------------------------------
#define SCAN_T 256
#define SCAN_ITEMS 8
#define SCAN_TILE (SCAN_T * SCAN_ITEMS)

template <typename T>
__device__ __forceinline__ uint64_t block_exclusive(uint64_t v, uint64_t *sh, uint64_t &total) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_T; o <<= 1) {
        const uint64_t a = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += a;
        __syncthreads();
    }
    total = sh[SCAN_T - 1];
    const uint64_t ex = sh[tid] - v;
    __syncthreads();
    return ex;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_T) k_scan_sums(const T *__restrict__ in, int64_t n, uint64_t *__restrict__ sums) {
    __shared__ uint64_t sh[SCAN_T];
    const int64_t b0 = (int64_t)blockIdx.x * SCAN_TILE;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t x = b0 + (int64_t)i * SCAN_T + threadIdx.x;
        if (x < n) s += (uint64_t)in[x];
    }
    uint64_t total = 0;
    block_exclusive<T>(s, sh, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename T, typename O>
__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const T *__restrict__ in, int64_t n,
                                                       const uint64_t *__restrict__ offs, O *__restrict__ out) {
    __shared__ uint64_t sh[SCAN_T];
    const int64_t b0 = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t x = b0 + i;
        v[i] = x < n ? in[x] : (T)0;
        s += (uint64_t)v[i];
    }
    uint64_t total = 0;
    uint64_t run = block_exclusive<T>(s, sh, total) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t x = b0 + i;
        if (x < n) out[x] = (O)run;
        run += (uint64_t)v[i];
    }
}

// out[i] = in[0] + ... + in[i - 1]; `work` holds scan_work_words(n) u64.
template <typename T, typename O>
void scan_exclusive(const T *in, O *out, int64_t n, uint64_t *work, hipStream_t st) {
    if (n <= 0) return;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        k_scan_apply<T, O><<<1, SCAN_T, 0, st>>>(in, n, nullptr, out);
        return;
    }
    uint64_t *sums = work, *offs = work + nb;
    k_scan_sums<T><<<(unsigned)nb, SCAN_T, 0, st>>>(in, n, sums);
    scan_exclusive<uint64_t, uint64_t>(sums, offs, nb, work + 2 * nb, st);
    k_scan_apply<T, O><<<(unsigned)nb, SCAN_T, 0, st>>>(in, n, offs, out);
}

int64_t scan_work_words(int64_t n) {
    int64_t w = 0;
    while (n > SCAN_TILE) {
        const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
        w += 2 * nb;
        n = nb;
    }
    return w + 2;
}

int64_t radix_temp_bytes(int64_t n, int key_bytes) {
    const int64_t nblocks = (n + SORT_TILE - 1) / SORT_TILE;
    const int64_t h = 256 * std::max<int64_t>(nblocks, 1);
    return 2 * h * 8 + scan_work_words(h) * 8 + n * (key_bytes + 4) + 256;
}

// Stable sort of (kin, vin) by the bits [0, end_bit) of the keys into (kout,
// vout); temp holds radix_temp_bytes(n, sizeof(K)) bytes.  Inputs are not
// modified.
template <typename K>
void radix_sort_pairs(const K *kin, K *kout, const uint32_t *vin, uint32_t *vout, int64_t n, int end_bit, void *temp,
                      hipStream_t st) {
    if (n <= 0) return;
    const int64_t nblocks = (n + SORT_TILE - 1) / SORT_TILE;
    const int64_t h = 256 * nblocks;
    uint64_t *hist = (uint64_t *)temp, *slot = hist + h, *work = slot + h;
    K *kt = (K *)(work + scan_work_words(h));
    uint32_t *vt = (uint32_t *)(kt + n);
    const int passes = std::max(1, (end_bit + 7) / 8);
    // ping-pong so that the last pass lands in (kout, vout)
    const K *ks = kin;
    const uint32_t *vs = vin;
    for (int p = 0; p < passes; p++) {
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        K *kd = to_out ? kout : kt;
        uint32_t *vd = to_out ? vout : vt;
        k_radix_hist<K><<<(unsigned)nblocks, SORT_T, 0, st>>>(ks, n, 8 * p, hist, nblocks);
        scan_exclusive<uint64_t, uint64_t>(hist, slot, h, work, st);
        k_radix_scatter<K><<<(unsigned)nblocks, SORT_T, 0, st>>>(ks, vs, n, 8 * p, slot, nblocks, kd, vd);
        ks = kd;
        vs = vd;
    }
}

template void radix_sort_pairs<uint32_t>(const uint32_t *, uint32_t *, const uint32_t *, uint32_t *, int64_t, int,
                                         void *, hipStream_t);
template void radix_sort_pairs<uint64_t>(const uint64_t *, uint64_t *, const uint32_t *, uint32_t *, int64_t, int,
                                         void *, hipStream_t);
template void scan_exclusive<uint32_t, uint32_t>(const uint32_t *, uint32_t *, int64_t, uint64_t *, hipStream_t);
template void scan_exclusive<uint64_t, uint64_t>(const uint64_t *, uint64_t *, int64_t, uint64_t *, hipStream_t);

}  // namespace sfe
