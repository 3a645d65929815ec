// ydrop_common.h -- device helpers shared by the gapped-extension kernels.
#pragma once
#include <type_traits>

#include "sfe_kernels.h"

namespace sfe {

#define NEG SFE_NEG

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imax3(int a, int b, int c) { return imax(imax(a, b), c); }

__device__ __forceinline__ int codeA(const SeqSetView &T, const HalfTask &tk, int64_t i) {
    if (i < 0 || i >= tk.nA) return 4;
    return base_code(T, tk.a0 + (int64_t)tk.adir * i);
}
__device__ __forceinline__ int codeB(const SeqSetView &Q, const HalfTask &tk, int64_t j) {
    if (j < 0 || j >= tk.nB) return 4;
    return base_code(Q, tk.b0 + (int64_t)tk.bdir * j);
}

// Cross-lane helpers (DPP): lane l receives lane l-1 (shr) or l+1 (shl); the
// lane without a source keeps `old`.
__device__ __forceinline__ int dpp_shr1(int old, int src) {
    return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_shl1(int old, int src) {
    return __builtin_amdgcn_update_dpp(old, src, 0x130, 0xf, 0xf, false);
}
// Maximum over the wave of values >= NEG (uniform result): row_shr 1, 2, 4, 8
// within each row of 16 lanes (lanes without a source see NEG), then
// row_bcast 15 and 31 carry row maxima into the rows above; lane 63 ends with
// the maximum.
__device__ __forceinline__ int wave_max_dpp(int v) {
    v = imax(v, __builtin_amdgcn_update_dpp(NEG, v, 0x111, 0xf, 0xf, false));
    v = imax(v, __builtin_amdgcn_update_dpp(NEG, v, 0x112, 0xf, 0xf, false));
    v = imax(v, __builtin_amdgcn_update_dpp(NEG, v, 0x114, 0xf, 0xf, false));
    v = imax(v, __builtin_amdgcn_update_dpp(NEG, v, 0x118, 0xf, 0xf, false));
    v = imax(v, __builtin_amdgcn_update_dpp(NEG, v, 0x142, 0xa, 0xf, false));
    v = imax(v, __builtin_amdgcn_update_dpp(NEG, v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, 63);
}

#define ROW_LIMIT (1 << 30)       // antidiagonals beyond this stop the half with HALF_SCORE_RANGE
#define RING 1024                 // sequence codes staged in LDS per side
#define RING_CHUNK 256            // codes loaded per refill

// Substitution scores.  PERM: every entry fits in int8, a row carries the
// packed scores of its target base against A, C, G, T (lo) and N (hi), and a
// query code travels as a v_perm selector picking its byte into bits 24..31.
// Otherwise rows carry the target code * 8 and the score is read from LDS.
template <bool PERM> struct Scorer;
template <> struct Scorer<true> {
    static __device__ __forceinline__ int bsel(int code) { return (code << 24) | 0x000c0c0c; }
    static __device__ __forceinline__ int score(int plo, int phi, int bsel, const int *) {
        return (int)__builtin_amdgcn_perm((uint32_t)phi, (uint32_t)plo, (uint32_t)bsel) >> 24;
    }
};
template <> struct Scorer<false> {
    static __device__ __forceinline__ int bsel(int code) { return code; }
    static __device__ __forceinline__ int score(int plo, int, int bsel, const int *sub) { return sub[plo + bsel]; }
};

// Loads codes of positions [from, from + RING_CHUNK) of one side of a half into
// its LDS ring of RS codes (index & (RS - 1)); positions outside [0, n) read as
// N.  All NT threads of the block take part (tid = thread index).  A ring must
// hold every position the band window can read: the window, its slide margin
// and one refill chunk.
template <int NT = 64, int RS = RING>
__device__ __forceinline__ void ring_fill(uint8_t *ring, const SeqSetView &S, int64_t p0, int64_t dir, int64_t n,
                                          int64_t from, int tid) {
    static_assert((RS & (RS - 1)) == 0 && RS >= RING_CHUNK, "ring size");
#pragma unroll 4
    for (int x = tid; x < RING_CHUNK; x += NT) {
        const int64_t j = from + x;
        int c = 4;
        if (j >= 0 && j < n) c = base_code(S, p0 + dir * j);
        ring[j & (RS - 1)] = (uint8_t)c;
    }
    __syncthreads();
}

}  // namespace sfe
