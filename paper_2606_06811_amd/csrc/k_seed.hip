// k_seed.hip -- packing, position table, seed hits and the ungapped X-drop
// filter on gfx950 (Sec. 1, Sec. 3, Sec. 7, Sec. 8 of the paper).
#include "sfe_kernels.h"

namespace sfe {

__constant__ uint8_t c_enc[256];   // bits 0-1 code, bit 2 N, bit 3 soft, bit 7 invalid letter

hipError_t upload_encoding_table(hipStream_t st) {
    uint8_t t[256];
    for (int c = 0; c < 256; c++) t[c] = 0x80;
    const char *N = "NRYSWKMBDHV";
    for (int s = 0; s < 2; s++) {
        int off = s ? 'a' - 'A' : 0;
        uint8_t soft = s ? 8 : 0;
        t['A' + off] = 0 | soft;
        t['C' + off] = 1 | soft;
        t['G' + off] = 2 | soft;
        t['T' + off] = 3 | soft;
        for (const char *p = N; *p; p++) t[*p + off] = 4 | soft;
    }
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_enc), t, 256, 0, hipMemcpyHostToDevice, st);
}

// One thread per 32 output bases.  rc = 1 writes the reverse complement.
__global__ void k_pack(const uint8_t *__restrict__ txt, int64_t len, int64_t out_start, int rc,
                       uint32_t *__restrict__ bases, uint32_t *__restrict__ nbits,
                       uint32_t *__restrict__ sbits, int *__restrict__ bad) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p0 = g * 32;
    if (p0 >= len) return;
    uint32_t w0 = 0, w1 = 0, nb = 0, sb = 0;
    int badl = 0;
    for (int u = 0; u < 32; u++) {
        int64_t p = p0 + u;
        if (p >= len) break;
        int64_t src = rc ? len - 1 - p : p;
        uint8_t e = c_enc[txt[src]];
        badl |= e >> 7;
        uint32_t isn = (e >> 2) & 1u;
        uint32_t code = isn ? 0u : (uint32_t)(e & 3u);
        if (rc && !isn) code = 3u - code;
        if (u < 16) w0 |= code << (2 * u); else w1 |= code << (2 * (u - 16));
        nb |= isn << u;
        sb |= (uint32_t)((e >> 3) & 1u) << u;
    }
    int64_t wp = (out_start + p0) >> 4;
    bases[wp] = w0;
    bases[wp + 1] = w1;
    nbits[(out_start + p0) >> 5] = nb;
    sbits[(out_start + p0) >> 5] = sb;
    if (badl) atomicOr(bad, 1);
}

// nsum bit x = N-plane word x is not zero (one ballot per 64 words; nsum zeroed before).
__global__ void k_nsum(const uint32_t *__restrict__ nbits, int64_t nwords, uint32_t *__restrict__ nsum) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t m = __ballot(x < nwords && nbits[x < nwords ? x : 0] != 0);
    if ((threadIdx.x & 63) == 0 && x < nwords) {
        nsum[x >> 5] = (uint32_t)m;
        nsum[(x >> 5) + 1] = (uint32_t)(m >> 32);
    }
}

// keys[x] = seed key of target window x*step, or `sentinel` when invalid.
__global__ void k_index_keys(SeqSetView T, int64_t nslots, int32_t step, SeedDesc sd, uint32_t sentinel,
                             uint32_t *__restrict__ keys, uint32_t *__restrict__ pos) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nslots) return;
    int64_t p = x * step;
    uint32_t key;
    bool ok = window_key(T, p, sd, &key);
    keys[x] = ok ? key : sentinel;
    pos[x] = (uint32_t)p;
}

// offsets[kk] = first index x with keys[x] >= kk, for kk in [0, K]; keys sorted.
__global__ void k_offsets(const uint32_t *__restrict__ keys, int64_t n, uint32_t K, uint32_t *__restrict__ offsets) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > n) return;
    int64_t prev = x > 0 ? (int64_t)keys[x - 1] : -1;
    int64_t cur = x < n ? (int64_t)keys[x] : (int64_t)K + 1;
    if (cur > (int64_t)K) cur = K;
    for (int64_t kk = prev + 1; kk <= cur; kk++) offsets[kk] = (uint32_t)x;
}

// ---------------------------------------------------------------------------
// Query windows: chunks of 64 consecutive windows of one (query, strand) unit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int seed_buckets(const SeqSetView &Q, int64_t p, const SeedDesc &sd,
                                            const uint32_t *__restrict__ offsets, uint32_t *bstart,
                                            uint32_t *bcount) {
    uint32_t key;
    if (!window_key(Q, p, sd, &key)) return 0;
    int nb = 0;
    int nvar = sd.transitions ? sd.weight : 0;
    for (int v = -1; v < nvar; v++) {
        uint32_t kk = key;
        if (v >= 0) kk ^= 2u << (2 * (sd.weight - 1 - v));
        uint32_t s = offsets[kk], e = offsets[kk + 1];
        bstart[nb] = s;
        bcount[nb] = e - s;
        nb++;
    }
    return nb;
}

__global__ void __launch_bounds__(64) k_seed_count(const UnitDesc *__restrict__ units, const Chunk *__restrict__ chunks,
                                                   SeqSetView Qp, SeqSetView Qm, const uint32_t *__restrict__ offsets,
                                                   SeedDesc sd, uint64_t *__restrict__ counts) {
    Chunk c = chunks[blockIdx.x];
    UnitDesc u = units[c.unit];
    int64_t q = (int64_t)c.w0 + threadIdx.x;
    uint64_t n = 0;
    if (q + sd.span <= u.len) {
        uint32_t bs[17], bc[17];
        int nb = seed_buckets(u.strand ? Qm : Qp, u.seq_start + q, sd, offsets, bs, bc);
        for (int b = 0; b < nb; b++) n += bc[b];
    }
    counts[(int64_t)blockIdx.x * 64 + threadIdx.x] = n;
}

// Writes the hits of each window at its offset, merged into t order.
__global__ void __launch_bounds__(64) k_seed_emit(const UnitDesc *__restrict__ units, const Chunk *__restrict__ chunks,
                                                  SeqSetView Qp, SeqSetView Qm, const uint32_t *__restrict__ offsets,
                                                  const uint32_t *__restrict__ tpos, SeedDesc sd,
                                                  const uint64_t *__restrict__ hit_off, sfe_hit *__restrict__ out) {
    Chunk c = chunks[blockIdx.x];
    UnitDesc u = units[c.unit];
    int64_t q = (int64_t)c.w0 + threadIdx.x;
    if (q + sd.span > u.len) return;
    uint32_t bs[17], bc[17];
    int nb = seed_buckets(u.strand ? Qm : Qp, u.seq_start + q, sd, offsets, bs, bc);
    uint64_t o = hit_off[(int64_t)blockIdx.x * 64 + threadIdx.x];
    // k-way merge of the (t-sorted) buckets; buckets hold disjoint t sets
    for (;;) {
        int bmin = -1;
        uint32_t tmin = 0xffffffffu;
        for (int b = 0; b < nb; b++) {
            if (bc[b]) {
                uint32_t t = tpos[bs[b]];
                if (bmin < 0 || t < tmin) { tmin = t; bmin = b; }
            }
        }
        if (bmin < 0) break;
        bs[bmin]++;
        bc[bmin]--;
        sfe_hit h;
        h.t = tmin;
        h.q = (uint32_t)q;
        h.query_id = (uint32_t)u.query_id;
        h.strand = (uint8_t)u.strand;
        h.pad[0] = h.pad[1] = h.pad[2] = 0;
        out[o++] = h;
    }
}

// ---------------------------------------------------------------------------
// Ungapped X-drop (one hit per lane)
// ---------------------------------------------------------------------------
struct XResult { int64_t t0, q0, len; int32_t score; int32_t work; bool range; };

// Codes of 16 consecutive bases starting at absolute position p of a set:
// bits 2u..2u+1 of c2 = base p + u (N stored as 0), bit u of n = base p + u
// is N.  Reads at most 46 bases past p + 15 (inside every sequence's padding).
struct Codes16 {
    uint32_t c2, n;
};
__device__ __forceinline__ Codes16 codes16(const SeqSetView &S, int64_t p) {
    const int64_t w = p >> 4;
    const int sh = (int)(p & 15) * 2;
    uint32_t c2 = S.bases[w];
    if (sh) c2 = (uint32_t)((((uint64_t)S.bases[w + 1] << 32) | c2) >> sh);
    const int64_t nw = p >> 5;
    const int nsh = (int)(p & 31);
    // the N plane is read only where its summary bits say it holds an N
    const uint32_t flags =
        (uint32_t)((((uint64_t)S.nsum[(nw >> 5) + 1] << 32) | S.nsum[nw >> 5]) >> (nw & 31)) & 3u;
    uint32_t n = 0;
    if (flags & 1u) n = S.nbits[nw] >> nsh;
    if (nsh > 16 && (flags & 2u)) n |= S.nbits[nw + 1] << (32 - nsh);
    return Codes16{c2, n};
}
__device__ __forceinline__ int code_at(const Codes16 &c, int u) {
    return ((c.n >> u) & 1u) ? 4 : (int)((c.c2 >> (2 * u)) & 3u);
}

// Tables of the ungapped filter in LDS: sub[a * 8 + b] for codes a, b in
// 0..4 (N = 4), and the 16 N-free pairs at (a << 2) | b, as int8 when every
// score fits (I8) or int32.
struct XTables {
    int sub[40];
    int sub16[16];
    int8_t sub8[16];
};

__device__ __forceinline__ void load_xtables(XTables &x, const ScoreDesc &sc) {
    const int i = threadIdx.x;
    if (i < 40) x.sub[i] = (i & 7) < 5 ? sc.sub[i >> 3][i & 7] : 0;
    if (i < 16) {
        x.sub16[i] = sc.sub[i >> 2][i & 3];
        x.sub8[i] = (int8_t)sc.sub[i >> 2][i & 3];
    }
}

template <bool I8>
__device__ __forceinline__ int pair_score(const XTables &x, uint32_t ca, uint32_t cb, int i) {
    const uint32_t idx = (((ca >> (2 * i)) & 3u) << 2) | ((cb >> (2 * i)) & 3u);
    return I8 ? (int)x.sub8[idx] : x.sub16[idx];
}

// Codes of a 16-base block in reverse order: the block of m <= 16 bases whose
// base u (u < m) becomes position m - 1 - u.
__device__ __forceinline__ Codes16 reverse16(Codes16 c, int m) {
    uint32_t r = __builtin_bitreverse32(c.c2);                      // field u -> 15 - u, its two bits swapped
    r = ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
    const uint32_t n = __builtin_bitreverse32(c.n & 0xffffu);        // bit u -> 31 - u
    return Codes16{r >> (2 * (16 - m)), n >> (32 - m)};
}

// Score of the seed span (span <= 32 columns from t, q).
template <bool I8>
__device__ __forceinline__ int32_t span_score(const SeqSetView &T, int64_t pt, const SeqSetView &Q, int64_t pq,
                                              int span, const XTables &x) {
    int32_t s0 = 0;
    for (int h = 0; h < span; h += 16) {
        const Codes16 a = codes16(T, pt + h), b = codes16(Q, pq + h);
        const int m = min(16, span - h);
        if (((a.n | b.n) & 0xffffu) == 0) {
#pragma unroll
            for (int i = 0; i < 16; i++)
                if (i < m) s0 += pair_score<I8>(x, a.c2, b.c2, i);
        } else {
            for (int i = 0; i < m; i++) s0 += x.sub[code_at(a, i) * 8 + code_at(b, i)];
        }
    }
    return s0;
}

// The 64 bases from absolute position p0 as four 16-base code words (N read
// as its stored code); reads the five words that hold them.
__device__ __forceinline__ void window64(const SeqSetView &S, int64_t p0, uint32_t X[4]) {
    const int64_t w = p0 >> 4;
    const uint32_t sh = (uint32_t)(p0 & 15) * 2;
    uint32_t W[5];
#pragma unroll
    for (int i = 0; i < 5; i++) W[i] = S.bases[w + i];
#pragma unroll
    for (int i = 0; i < 4; i++) X[i] = (uint32_t)((((uint64_t)W[i + 1] << 32) | W[i]) >> sh);
}

// True when no base of [p0, p0 + len) is N (len <= 64), from the summary bits
// of the N plane.
__device__ __forceinline__ bool window_has_no_n(const SeqSetView &S, int64_t p0, int len) {
    const int64_t nw0 = p0 >> 5, nw1 = (p0 + len - 1) >> 5;
    const uint64_t bits = ((uint64_t)S.nsum[(nw0 >> 5) + 1] << 32) | S.nsum[nw0 >> 5];
    const uint32_t cnt = (uint32_t)(nw1 - nw0 + 1);
    return ((bits >> (nw0 & 31)) & ((1ull << cnt) - 1)) == 0;
}

// Ungapped X-drop of one hit (t, q relative to their sequences, which start
// at tb / qb in their sets and have lengths nt / nq): the seed span, then the
// scan to the right of it and the scan to the left, each stopping at the first
// column where best - running > X (a strictly better running score moves the
// end; the sequence ends stop it too).  The two scans run in one loop of
// 16-column blocks, so a lane whose right scan ends early starts its left scan
// while the other lanes of its wave are still scanning right.  A block without
// N takes the unrolled path (pair scores from the 16-entry table, the stop
// rule applied column by column through a live flag); the last, partial block
// of a scan and blocks with an N take the column loop.  work counts the
// columns scored, the span included.
template <bool I8>
__device__ __forceinline__ XResult xdrop_hit(const SeqSetView &T, int64_t tb, int64_t nt, const SeqSetView &Q,
                                             int64_t qb, int64_t nq, int64_t t, int64_t q, int span,
                                             const XTables &x, int32_t X) {
    int64_t lim = min(nt - t - span, nq - q - span);
    // Most hits end within the first block on each side: when both first blocks are whole
    // and no base from t - 16 to the end of the first right block is N, one round of loads
    // (64 bases of each sequence from t - 16, q - 16) serves the span and both first blocks.
    const bool pre = span < 32 && lim >= 16 && t >= 16 && q >= 16 && window_has_no_n(T, tb + t - 16, span + 32) &&
                     window_has_no_n(Q, qb + q - 16, span + 32);
    Codes16 ra{0, 0}, rb{0, 0}, la{0, 0}, lb{0, 0};
    int32_t s0 = 0;
    if (pre) {
        uint32_t A[4], B[4];
        window64(T, tb + t - 16, A);
        window64(Q, qb + q - 16, B);
#pragma unroll
        for (int i = 0; i < 32; i++)
            if (i < span) s0 += pair_score<I8>(x, A[1 + i / 16], B[1 + i / 16], i & 15);
        // first right block: bases t + span .. t + span + 15 (span < 32), from A[1..3]
        const uint32_t sh = 2u * (uint32_t)(span & 15);
        const int k = 1 + span / 16;
        const uint32_t a0 = k == 1 ? A[1] : A[2], a1 = k == 1 ? A[2] : A[3];
        const uint32_t b0 = k == 1 ? B[1] : B[2], b1 = k == 1 ? B[2] : B[3];
        ra.c2 = (uint32_t)((((uint64_t)a1 << 32) | a0) >> sh);
        rb.c2 = (uint32_t)((((uint64_t)b1 << 32) | b0) >> sh);
        la.c2 = A[0];       // bases t - 16 .. t - 1, reversed below like any left block
        lb.c2 = B[0];
    } else {
        s0 = span_score<I8>(T, tb + t, Q, qb + q, span, x);
    }
    int32_t work = span;
    bool range = false;
    int side = 0;                                   // 0 right, 1 left
    int64_t r0 = 1, arg = 0, R = 0;
    int32_t s = 0, best = 0, bR = 0;
    for (;;) {
        const int64_t left = lim - r0 + 1;        // columns not yet scanned on this side
        bool done = left <= 0;
        if (!done) {
            const int m = (int)min((int64_t)16, left);
            // right: bases t + span - 1 + r of both; left: t - r, read as the block ending at t - r0
            Codes16 a, b;
            if (pre && r0 == 1 && m == 16) {
                a = side ? la : ra;
                b = side ? lb : rb;
            } else {
                const int64_t pt = side ? tb + t - r0 - m + 1 : tb + t + span - 1 + r0;
                const int64_t pq = side ? qb + q - r0 - m + 1 : qb + q + span - 1 + r0;
                a = codes16(T, pt);
                b = codes16(Q, pq);
            }
            if (side) {
                a = reverse16(a, m);
                b = reverse16(b, m);
            }
            const int32_t best0 = best;
            int argi = 0;
            bool live = true;
            if (m == 16 && ((a.n | b.n) & 0xffffu) == 0) {
                int sv[16];
#pragma unroll
                for (int i = 0; i < 16; i++) sv[i] = pair_score<I8>(x, a.c2, b.c2, i);
#pragma unroll
                for (int i = 0; i < 16; i++) {
                    s += sv[i];
                    work += live ? 1 : 0;
                    const bool up = live && s > best;
                    best = up ? s : best;
                    argi = up ? i : argi;
                    live = live && best - s <= X;
                }
            } else {
                for (int i = 0; i < m && live; i++) {
                    s += x.sub[code_at(a, i) * 8 + code_at(b, i)];
                    work++;
                    if (s > best) { best = s; argi = i; }
                    else if (best - s > X) live = false;
                }
            }
            if (best > best0) arg = r0 + argi;
            range = best >= SFE_SCORE_LIMIT;
            r0 += 16;
            done = !live || range || m < 16;
        }
        if (done) {
            if (side == 0 && !range) {
                bR = best;
                R = arg;
                side = 1;
                lim = min(t, q);
                r0 = 1;
                s = best = 0;
                arg = 0;
                continue;
            }
            break;
        }
    }
    XResult res;
    if (side == 0) { bR = best; R = arg; best = 0; arg = 0; }   // stopped by the score range on the right
    res.t0 = t - arg;
    res.q0 = q - arg;
    res.len = arg + span + R;
    res.score = s0 + best + bR;
    res.work = work;
    res.range = range;
    return res;
}

template <bool I8>
__global__ void k_xdrop_raw(const sfe_hit *__restrict__ hits, int64_t n, const QueryDesc *__restrict__ qd,
                            int32_t nq, SeqSetView T, int64_t tb, int64_t nt, SeqSetView Qp, SeqSetView Qm,
                            ScoreDesc sc, int span, sfe_hsp *__restrict__ out, int *__restrict__ err) {
    __shared__ XTables xt;
    load_xtables(xt, sc);
    __syncthreads();
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    sfe_hit h = hits[x];
    QueryDesc d = qd[h.query_id];
    XResult r = xdrop_hit<I8>(T, tb, nt, h.strand ? Qm : Qp, d.start, d.len, h.t, h.q, span, xt, sc.xdrop);
    if (r.range) atomicOr(err, 1);
    sfe_hsp o;
    o.t0 = (uint32_t)r.t0;
    o.q0 = (uint32_t)r.q0;
    o.len = (uint32_t)r.len;
    o.score = r.score;
    o.query_id = h.query_id;
    o.strand = h.strand;
    o.pad[0] = o.pad[1] = o.pad[2] = 0;
    out[x] = o;
}

// Fused seed + X-drop: a block takes one chunk of 64 windows; its threads
// walk the chunk's hits (flattened over windows and buckets) and append the
// passing segments.  Hits never leave the chip.  The kernel waits on gathers
// most of the time, so it asks for 8 waves per SIMD (64 VGPRs, with 160 bytes
// per lane spilled to scratch): ~10 % faster than the 7 waves its 71 VGPRs
// would allow.
template <bool I8>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) k_seed_xdrop(const UnitDesc *__restrict__ units, const Chunk *__restrict__ chunks,
                                                    SeqSetView T, int64_t tb, int64_t nt, SeqSetView Qp, SeqSetView Qm,
                                                    const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ tpos,
                                                    SeedDesc sd, ScoreDesc sc, sfe_hsp *__restrict__ out, uint64_t cap,
                                                    unsigned long long *__restrict__ counters) {
    __shared__ XTables xt;
    __shared__ uint32_t s_bstart[64][16];
    __shared__ uint32_t s_bcum[64][17];     // cumulative bucket counts per window
    __shared__ uint32_t s_wcum[65];         // cumulative hit counts over windows
    Chunk c = chunks[blockIdx.x];
    UnitDesc u = units[c.unit];
    const SeqSetView Q = u.strand ? Qm : Qp;
    load_xtables(xt, sc);
    if (threadIdx.x < 64) {
        int64_t q = (int64_t)c.w0 + threadIdx.x;
        uint32_t bs[17], bc[17];
        int nb = 0;
        if (q + sd.span <= u.len) nb = seed_buckets(Q, u.seq_start + q, sd, offsets, bs, bc);
        uint32_t cum = 0;
        s_bcum[threadIdx.x][0] = 0;
        for (int b = 0; b < 16; b++) {
            uint32_t cnt = b < nb ? bc[b] : 0;
            s_bstart[threadIdx.x][b] = b < nb ? bs[b] : 0;
            cum += cnt;
            s_bcum[threadIdx.x][b + 1] = cum;
        }
        s_wcum[threadIdx.x + 1] = cum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_wcum[0] = 0;
        for (int w = 1; w <= 64; w++) s_wcum[w] += s_wcum[w - 1];
    }
    __syncthreads();
    uint32_t total = s_wcum[64];
    if (threadIdx.x == 0 && total) atomicAdd(&counters[0], (unsigned long long)total);
    unsigned long long work = 0;
    for (uint32_t h = threadIdx.x; h < total; h += blockDim.x) {
        // window: last w with s_wcum[w] <= h
        int lo = 0, hi = 63;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (s_wcum[mid] <= h) lo = mid; else hi = mid - 1;
        }
        int w = lo;
        uint32_t r = h - s_wcum[w];
        int b = 0;
        while (s_bcum[w][b + 1] <= r) b++;
        uint32_t t = tpos[s_bstart[w][b] + (r - s_bcum[w][b])];
        int64_t q = (int64_t)c.w0 + w;
        XResult x = xdrop_hit<I8>(T, tb, nt, Q, u.seq_start, u.len, t, q, sd.span, xt, sc.xdrop);
        work += (unsigned long long)x.work;
        if (x.range) atomicOr((unsigned long long *)&counters[3], 1ull);
        if (x.score >= sc.hsp_thresh) {
            unsigned long long slot = atomicAdd(&counters[1], 1ull);
            if (slot < cap) {
                sfe_hsp o;
                o.t0 = (uint32_t)x.t0;
                o.q0 = (uint32_t)x.q0;
                o.len = (uint32_t)x.len;
                o.score = x.score;
                o.query_id = (uint32_t)u.query_id;
                o.strand = (uint8_t)u.strand;
                o.pad[0] = o.pad[1] = o.pad[2] = 0;
                out[slot] = o;
            }
        }
    }
    // columns scored, summed over the wave, one atomic per wave
    for (int m = 32; m >= 1; m >>= 1) work += __shfl_xor(work, m, 64);
    if ((threadIdx.x & 63) == 0 && work) atomicAdd(&counters[2], work);
}

bool scores_fit_int8(const ScoreDesc &sc) {
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            if (sc.sub[a][b] < -128 || sc.sub[a][b] > 127) return false;
    return true;
}

void launch_xdrop_raw(const sfe_hit *hits, int64_t n, const QueryDesc *qd, int32_t nq, SeqSetView T, int64_t tb,
                      int64_t nt, SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc, int span, sfe_hsp *out, int *err,
                      hipStream_t st) {
    if (n <= 0) return;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (scores_fit_int8(sc))
        k_xdrop_raw<true><<<g, 256, 0, st>>>(hits, n, qd, nq, T, tb, nt, Qp, Qm, sc, span, out, err);
    else
        k_xdrop_raw<false><<<g, 256, 0, st>>>(hits, n, qd, nq, T, tb, nt, Qp, Qm, sc, span, out, err);
}

void launch_seed_xdrop(const UnitDesc *units, const Chunk *chunks, int64_t nch, SeqSetView T, int64_t tb, int64_t nt,
                       SeqSetView Qp, SeqSetView Qm, const uint32_t *offsets, const uint32_t *tpos, const SeedDesc &sd,
                       const ScoreDesc &sc, sfe_hsp *out, uint64_t cap, unsigned long long *counters, hipStream_t st) {
    if (nch <= 0) return;
    if (scores_fit_int8(sc))
        k_seed_xdrop<true><<<(unsigned)nch, 256, 0, st>>>(units, chunks, T, tb, nt, Qp, Qm, offsets, tpos, sd, sc, out,
                                                          cap, counters);
    else
        k_seed_xdrop<false><<<(unsigned)nch, 256, 0, st>>>(units, chunks, T, tb, nt, Qp, Qm, offsets, tpos, sd, sc,
                                                           out, cap, counters);
}

// ---------------------------------------------------------------------------
// HSP set helpers: field extraction for the LSD multi-key sort, gather,
// duplicate flags.
// ---------------------------------------------------------------------------
__global__ void k_hsp_key(const sfe_hsp *__restrict__ h, const uint32_t *__restrict__ perm, int64_t n, int field,
                          uint32_t *__restrict__ key) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    sfe_hsp r = h[perm[x]];
    uint32_t k;
    switch (field) {
    case 0: k = r.len; break;
    case 1: k = r.q0; break;
    case 2: k = r.t0; break;
    case 3: k = r.strand; break;
    case 4: k = ~((uint32_t)r.score ^ 0x80000000u); break;   // score descending
    default: k = r.query_id; break;
    }
    key[x] = k;
}

__global__ void k_iota(uint32_t *__restrict__ a, int64_t n) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) a[x] = (uint32_t)x;
}

__global__ void k_hsp_unique_flags(const sfe_hsp *__restrict__ h, const uint32_t *__restrict__ perm, int64_t n,
                                   uint32_t *__restrict__ flag) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    uint32_t f = 1;
    if (x > 0) {
        sfe_hsp a = h[perm[x - 1]], b = h[perm[x]];
        f = !(a.t0 == b.t0 && a.q0 == b.q0 && a.len == b.len && a.strand == b.strand && a.query_id == b.query_id);
    }
    flag[x] = f;
}

__global__ void k_hsp_compact(const sfe_hsp *__restrict__ h, const uint32_t *__restrict__ perm,
                              const uint32_t *__restrict__ flag, const uint32_t *__restrict__ dst, int64_t n,
                              sfe_hsp *__restrict__ out) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    if (flag[x]) out[dst[x]] = h[perm[x]];
}

}  // namespace sfe
