// sfe_internal.h -- shared definitions of the gfx950 library (not installed).
//
// Device layout of a sequence set (target, query plus strands, query minus
// strands): every sequence starts at a multiple of 64 bases and is followed by
// at least 64 bases of padding, so word-granular reads never leave the
// buffers.  Per base p of the set:
//   bases[p >> 4] bits 2*(p & 15) .. +1   code A0 C1 G2 T3 (N stored as 0)
//   nbits[p >> 5] bit  p & 31             1 = N (or an IUPAC ambiguity letter)
//   sbits[p >> 5] bit  p & 31             1 = soft-masked (lower case)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sfe.h"

#define SFE_NEG (-(1 << 30))
#define SFE_SCORE_LIMIT (1 << 29)   // a score this large is reported as SFE_ERANGE

namespace sfe {

struct SeqSetView {
    const uint32_t *bases;
    const uint32_t *nbits;
    const uint32_t *sbits;
    const uint32_t *nsum;   // bit x set when N-plane word x (bases 32x .. 32x + 31) holds an N
};

// code 0..3, or 4 for N
__device__ __forceinline__ int base_code(const SeqSetView &s, int64_t p) {
    uint32_t w = s.bases[p >> 4];
    uint32_t n = s.nbits[p >> 5];
    int c = (int)((w >> ((p & 15) * 2)) & 3u);
    return ((n >> (p & 31)) & 1u) ? 4 : c;
}

// Seed description resolved on the host.
struct SeedDesc {
    int32_t span, weight, transitions, step;
    int32_t care[16];
};

// 64 consecutive bases starting at p (bit 2*u = base p+u) as two words, and
// the OR of the N and soft planes over 32 bases starting at p.
__device__ __forceinline__ uint64_t bases64(const SeqSetView &s, int64_t p) {
    int64_t w = p >> 4;
    int sh = (int)(p & 15) * 2;
    uint64_t lo = (uint64_t)s.bases[w] | ((uint64_t)s.bases[w + 1] << 32);
    uint64_t hi = (uint64_t)s.bases[w + 2];
    if (sh == 0) return lo;
    return (lo >> sh) | (hi << (64 - sh));
}
__device__ __forceinline__ uint32_t masked32(const SeqSetView &s, int64_t p) {
    int64_t w = p >> 5;
    int sh = (int)(p & 31);
    uint64_t a = (uint64_t)(s.nbits[w] | s.sbits[w]) | ((uint64_t)(s.nbits[w + 1] | s.sbits[w + 1]) << 32);
    return (uint32_t)(a >> sh);
}

// Window at p (absolute position in the set) of a sequence whose last valid
// window start is `last`: valid iff p <= last and no N / soft-masked base in
// the span.  On success *key holds the care codes, first care position most
// significant.
__device__ __forceinline__ bool window_key(const SeqSetView &s, int64_t p, const SeedDesc &sd, uint32_t *key) {
    uint32_t m = masked32(s, p);
    uint32_t spanmask = sd.span >= 32 ? 0xffffffffu : ((1u << sd.span) - 1u);
    if (m & spanmask) return false;
    uint64_t b = bases64(s, p);
    uint32_t k = 0;
    for (int c = 0; c < sd.weight; c++) k = (k << 2) | (uint32_t)((b >> (2 * sd.care[c])) & 3u);
    *key = k;
    return true;
}

// ---------------------------------------------------------------------------
// Gapped extension: tasks, results, traceback arena
// ---------------------------------------------------------------------------
// A half reads A(i) = target[a0 + adir * i] for i < nA and
// B(j) = qset[b0 + bdir * j] for j < nB (positions absolute in their sets).
struct HalfTask {
    int64_t a0, b0;
    int64_t nA, nB;
    int32_t adir, bdir;
    int32_t qset;           // 0 plus-strand query set, 1 minus-strand set
    int32_t pad;
};

#define HALF_OK 0
#define HALF_WIDTH_OVERFLOW 1
#define HALF_ARENA_OVERFLOW 2
#define HALF_SCORE_RANGE 3      // a score reached 2^29 (or the band 2^30 antidiagonals)
#define HALF_RUNS_OVERFLOW 4    // the run arena is full
#define HALF_TRACE_ERROR 5      // traceback codes inconsistent (internal error)
#define HALF_LONG 7             // reached the antidiagonal cap of its launch (re-run by a wave group)

struct HalfResult {
    int32_t best, i_end, j_end, status;
    uint64_t cells;
    // workgroup kernel: device address of the allocation holding the end
    // cell's record, and the record's offset in it; fused kernel: first run
    // in the run arena, and the number of runs
    uint64_t tb_page;
    uint32_t tb_end;
    int32_t k_last;         // last antidiagonal computed
};

// Chunk pool of the fused kernels: `nchunks` chunks of 2^shift bytes at base,
// bit c of bits[] set while chunk c is held by a half.  A half keeps its
// traceback codes in a backward-linked chain of chunks, each laid out as
//   header (16 bytes): u32 previous chunk of the chain (~0 for the first),
//     u32 k0 = antidiagonal of its first record, u32 bytes of records used,
//     u32 scratch (the extension kernels' lanes outside a record store there);
//   records upward from offset 16, one per antidiagonal: one u32 of 4-bit
//     codes per lane group of G rows covering the computed range (row
//     r0 + w*G + x in bits 4x .. 4x+3 of word w; the 16-bit kernel's layout
//     is described with its decoder);
//   index downward from the end: the uint2 at 2^shift - 8*(x+1) holds
//     (offset of the record of antidiagonal k0 + x, its first row r0).
// Code bits as in the arena above.  Edit runs being traced go to a second
// chain (header u32 previous chunk, runs from offset 16).
struct ChunkPool {
    uint8_t *base;
    uint32_t *bits;
    int32_t *avail;         // free chunks not yet reserved
    int32_t nwords;         // nchunks / 32
    int32_t shift;
};

// Edit runs of traced halves (u32 len << 2 | op), handed out by a device counter.
struct RunArena {
    uint32_t *base;
    uint64_t cap;           // in runs
    unsigned long long *head;
};

// Halves ids[0 .. n) (or 0 .. n with ids null), claimed in order through *head.
struct WorkQueue {
    const int32_t *ids;
    int64_t n;
    unsigned int *head;
    const int64_t *n_dev;   // if set, the number of halves is *n_dev (read when the kernel starts)
};

// Traceback pointer arena.  Allocations of one or more ARENA_PAGE pages, a
// half's allocations chained backwards.  Allocation layout:
//   header (16 bytes): u64 device address of the half's previous allocation
//     (~0 for its first), u32 k0 = antidiagonal of the first record in this
//     allocation, u32 pages;
//   records upward from offset 16, one per antidiagonal k0, k0+1, ...:
//     u32 r0, u32 (g | G << 24), then g u32 words; word w holds the 4-bit codes
//     of rows r0 + w*G .. r0 + w*G + G-1 (G <= 8, row r0 + w*G + x in bits
//     4x .. 4x+3);
//   index downward from the end: u32 at size - 4*(x+1) = offset of the record
//     of antidiagonal k0 + x.
// Code bits: 0-1 H source (0 diagonal, 1 E, 2 F), 2 E opened from H,
//            3 F opened from H.
#define ARENA_PAGE 32768u
#define ARENA_HDR 16u

struct Arena {
    uint8_t *base;
    uint64_t bytes;
    unsigned long long *head;   // device counter: bytes handed out
};

__host__ __device__ __forceinline__ uint32_t rec_head_word(uint32_t groups, uint32_t G) { return groups | (G << 24); }

}  // namespace sfe
