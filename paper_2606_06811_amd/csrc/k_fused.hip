// k_fused.hip -- gapped Y-drop extension of anchor halves fused with their
// traceback, one 64-lane wave per half (Sec. 8 of the paper).
//
// The DP is the one described at the top of k_extend.hip.  The traceback
// codes of a half (one record per antidiagonal: one u32 of 4-bit codes per
// lane group of G rows, located through an index entry holding the record's
// offset and first row) go to a chain of fixed-size chunks taken from a pool
// shared by all waves.  When the half stops, the same wave walks the codes
// back from the end cell a run at a time, returning each chunk to the pool
// once the walk has left it; the run-length edit operations go to a second
// chain and are finally copied, contiguous, to the run arena.  The
// device thus holds codes only for the halves in flight, and a half never
// has to be re-run because its traceback is long -- only when the whole pool
// is exhausted.
//
// Work sources:
//  * plain (one block per half, the paper's mapping): block b runs half ids[b];
//  * persistent: a fixed grid of waves pulls halves from a queue (an atomic
//    head over `ids`) until it is empty.
#include "ydrop_common.h"

namespace sfe {

#define TB_IDX 512            // index entries staged in LDS during traceback

// Takes a free chunk (wave-uniform; -1 if none came free in time).  A wave
// first reserves one of the `avail` free chunks -- when none is left it
// sleeps and retries for a bounded time, as other waves return chunks -- and
// then looks for a clear bit: lanes read 64 bitmap words at once, lane 0
// claims the first clear bit seen.  A reservation guarantees a clear bit
// exists (a release clears its bit before it increments avail).  The fence
// after a claim (and before a release) orders the chunk's previous contents
// against its new owner across the L2s of the chip.
__device__ __forceinline__ int pool_alloc(const ChunkPool &p, int &hint, int lane) {
    bool reserved = false;
    for (int wait = 0; wait < 8192; wait++) {
        int got = 0;
        if (lane == 0) {
            got = atomicSub(p.avail, 1) > 0;
            if (!got) atomicAdd(p.avail, 1);
        }
        if (__builtin_amdgcn_readfirstlane(got)) { reserved = true; break; }
        __builtin_amdgcn_s_sleep(127);
    }
    if (!reserved) return -1;
    for (int t = 0; t < (1 << 20); t++) {
        const int w = (hint + lane) % p.nwords;
        const uint32_t word = __hip_atomic_load(&p.bits[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t m = __ballot(word != 0xffffffffu);
        if (!m) {
            hint = (hint + 64) % p.nwords;
            continue;
        }
        const int L = __builtin_ctzll(m);
        const int wl = __builtin_amdgcn_readlane(w, L);
        const uint32_t wd = (uint32_t)__builtin_amdgcn_readlane((int)word, L);
        const uint32_t bit = 1u << __builtin_ctz(~wd);
        uint32_t old = 0;
        if (lane == 0) old = atomicOr(&p.bits[wl], bit);
        old = (uint32_t)__builtin_amdgcn_readfirstlane((int)old);
        hint = wl;
        if (!(old & bit)) {
            __threadfence();
            return wl * 32 + __builtin_ctz(bit);
        }
    }
    if (lane == 0) atomicAdd(p.avail, 1);     // not reached while reservations hold
    return -1;
}

__device__ __forceinline__ void pool_free(const ChunkPool &p, int c, int lane) {
    __threadfence();
    if (lane == 0) {
        atomicAnd(&p.bits[c >> 5], ~(1u << (c & 31)));
        __threadfence();
        atomicAdd(p.avail, 1);
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ uint8_t *chunk_ptr(const ChunkPool &p, int c) {
    return p.base + ((uint64_t)(uint32_t)c << p.shift);
}
__device__ __forceinline__ uint32_t chunk_hdr(const ChunkPool &p, int c, int w) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)((const uint32_t *)chunk_ptr(p, c))[w]);
}
// Returns a backward-linked chain of chunks to the pool.
__device__ __forceinline__ void free_chain(const ChunkPool &p, int c, int lane) {
    for (int guard = 0; c >= 0 && guard < (1 << 24); guard++) {
        const int prev = (int)chunk_hdr(p, c, 0);
        pool_free(p, c, lane);
        c = prev;
    }
}

// Code of row r of a 16-bit record word (rows in pairs (p, p + P), pair p's
// nibbles at bits 12 - 4p (row p) and 28 - 4p (row p + P); nibble bits, high
// to low: from a gap, from F rather than E, E extended, F extended), in the
// layout of the 32-bit kernel (bits 0-1: 0 diagonal, 1 E, 2 F; bit 2: E
// opened from H; bit 3: F opened from H).
__device__ __forceinline__ uint32_t narrow_code(uint32_t w, uint32_t r, uint32_t P) {
    const uint32_t n = (w >> (r < P ? 12u - 4u * r : 28u - 4u * (r - P))) & 15u;
    return ((n & 8u) ? ((n & 4u) ? 2u : 1u) : 0u) | ((n & 2u) ? 0u : 4u) | ((n & 1u) ? 0u : 8u);
}

// Traceback of one half by one wave, a run at a time: from the current cell,
// lane l fetches the code of the l-th cell along the current direction
// (diagonal in state H, left in E, up in F) and one ballot finds where the
// run ends (an H cell not reached diagonally, a gap opened from H), so a run
// of up to 64 operations costs one index lookup in LDS and one code load per
// lane.  Index entries of the chunk being walked are staged in LDS 512
// antidiagonals at a time; a chunk goes back to the pool once the walk has
// left it.  The edit runs (end cell first) go to a chain of pool chunks, then
// to an exact-size slice of the run arena.  G = rows per code word of the
// records; NARROW selects the code layout of the 16-bit kernel (see
// narrow_code).  Frees every chunk it was given; returns the half's status.
template <bool NARROW>
__device__ int trace_half(const ChunkPool &pool, int &hint, int lane, int cur, int bi, int bj, int G,
                          const RunArena &ra, uint2 *tb_idx, uint64_t &run_off, uint32_t &nruns) {
    const uint32_t CH = 1u << pool.shift;
    const uint32_t RC = (CH - 16) / 4;           // runs per chunk of the run chain
    int status = HALF_OK;
    uint8_t *cb = nullptr;
    int k0 = 0;
    uint32_t fill = 0;
    wave_sync();
    const int64_t kk0 = (int64_t)bi + bj;
    bool bad = false, oom = false;
    // chunks holding only antidiagonals past the end cell go back at once
    while (cur >= 0 && (int64_t)chunk_hdr(pool, cur, 1) > kk0) {
        const int pc = (int)chunk_hdr(pool, cur, 0);
        pool_free(pool, cur, lane);
        cur = pc;
    }
    if (cur < 0) bad = true;
    else { cb = chunk_ptr(pool, cur); k0 = (int)chunk_hdr(pool, cur, 1); fill = chunk_hdr(pool, cur, 2); }
    int rcur = -1;
    uint32_t rfill = RC, cnt = 0;
    auto emit = [&](uint32_t w) {
        if (rfill == RC) {
            const int nc = pool_alloc(pool, hint, lane);
            if (nc < 0) return false;
            if (lane == 0) ((uint32_t *)chunk_ptr(pool, nc))[0] = (uint32_t)rcur;
            rcur = nc;
            rfill = 0;
        }
        if (lane == 0) ((uint32_t *)(chunk_ptr(pool, rcur) + 16))[rfill] = w;
        rfill++;
        cnt++;
        return true;
    };
    uint32_t cur_op = 0xffffffffu, cur_len = 0;
    // appends len operations op, closing the previous run when op changes
    auto push = [&](uint32_t op, uint32_t len) {
        if (len == 0) return;
        if (op == cur_op) { cur_len += len; return; }
        if (cur_len) {
            if (cnt >= (uint32_t)kk0) { bad = true; return; }    // runs <= operations <= bi + bj
            if (!emit((cur_len << 2) | cur_op)) { oom = true; return; }
        }
        cur_op = op;
        cur_len = len;
    };
    int64_t ic = -1;                  // antidiagonal of tb_idx[0] (-1: nothing staged)
    int ti = bi, tj = bj, st = 0;     // st: 0 H, 1 E (op I), 2 F (op D)
    int64_t guard = 2 * kk0 + 64;
    while (!bad && !oom && !(ti == 0 && tj == 0 && st == 0)) {
        if (--guard < 0 || (st == 1 && tj == 0) || (st == 2 && ti == 0)) { bad = true; break; }
        const int64_t kk = (int64_t)ti + tj;
        while (kk < k0) {             // the walk left this chunk
            const int pc = (int)chunk_hdr(pool, cur, 0);
            pool_free(pool, cur, lane);
            cur = pc;
            if (cur < 0) break;
            cb = chunk_ptr(pool, cur);
            k0 = (int)chunk_hdr(pool, cur, 1);
            fill = chunk_hdr(pool, cur, 2);
            ic = -1;
        }
        if (cur < 0) { bad = true; break; }
        const int64_t lowest = kk - (st == 0 ? 126 : 63);     // deepest antidiagonal of this round
        if (ic < 0 || (lowest < ic && ic > k0)) {
            ic = max((int64_t)k0, kk - TB_IDX + 1);
            wave_sync();
            for (int q = lane; q < TB_IDX; q += 64) {
                const int64_t kq = ic + q;
                tb_idx[q] = kq <= kk ? *(const uint2 *)(cb + CH - 8u * (uint32_t)(kq - k0 + 1)) : make_uint2(0u, 0u);
            }
            wave_sync();
        }
        // this lane's cell
        const int ci = st == 1 ? ti : ti - lane;
        const int cj = st == 2 ? tj : tj - lane;
        const int64_t ka = (int64_t)ci + cj;
        // (a gap state never reaches row or column 0: its run stops before)
        bool inside = ci >= (st == 2 ? 1 : 0) && cj >= (st == 1 ? 1 : 0) && ka >= 1 && ka >= ic && ka <= kk;
        // its code, when the cell lies in the computed range of its antidiagonal
        // (lanes past the end of the run may fall outside: that only stops the run)
        uint32_t code = 0;
        bool valid = false;
        if (inside) {
            const uint2 ent = tb_idx[ka - ic];
            if ((uint32_t)ci >= ent.y) {
                const uint32_t idx = (uint32_t)ci - ent.y;
                const uint64_t wofs = (uint64_t)ent.x + 4ull * (idx / (uint32_t)G);
                if (wofs + 4 <= (uint64_t)fill) {
                    valid = true;
                    const uint32_t w = *(const uint32_t *)(cb + wofs);
                    code = NARROW ? narrow_code(w, idx % (uint32_t)G, (uint32_t)G / 2)
                                  : (w >> (4u * (idx % (uint32_t)G))) & 15u;
                }
            }
        }
        if (st == 0) {
            // diagonal run: lanes 0 .. f-1 are M columns; lane f stops it
            const uint64_t stop = __ballot(!valid || (code & 3u) != 0);
            const int f = stop ? __builtin_ctzll(stop) : 64;
            push(0u, (uint32_t)f);
            ti -= f;
            tj -= f;
            if (f < 64 && !(ti == 0 && tj == 0)) {
                const uint32_t cf = (uint32_t)__builtin_amdgcn_readlane((int)code, f);
                const int fin = __builtin_amdgcn_readlane((int)inside, f);
                const int fva = __builtin_amdgcn_readlane((int)valid, f);
                if (fin && !fva) { bad = true; break; }      // the path needs a cell never computed
                if (fva) {
                    const uint32_t src = cf & 3u;
                    if (src == 3u) { bad = true; break; }
                    st = (int)src;
                }
            }
        } else {
            // gap run: every cell emits one gap column; the first cell whose gap
            // was opened from H ends it (and the walk returns to H)
            const uint32_t obit = st == 1 ? 4u : 8u;
            const uint64_t open = __ballot(valid && (code & obit) != 0);
            const uint64_t out = __ballot(!valid);
            const int fo = open ? __builtin_ctzll(open) : 64;
            const int fx = out ? __builtin_ctzll(out) : 64;
            const uint32_t op = st == 1 ? 1u : 2u;
            int len;
            if (fo < fx) {
                len = fo + 1;
                st = 0;
            } else {
                len = fx;
                if (fx < 64 && __builtin_amdgcn_readlane((int)inside, fx)) { bad = true; break; }
            }
            push(op, (uint32_t)len);
            if (op == 1u) tj -= len;
            else ti -= len;
        }
    }
    if (!bad && !oom && cur_len) {
        if (cnt >= (uint32_t)kk0) bad = true;
        else if (!emit((cur_len << 2) | cur_op)) oom = true;
    }
    if (bad) status = HALF_TRACE_ERROR;
    else if (oom) status = HALF_ARENA_OVERFLOW;
    if (status == HALF_OK) {
        unsigned long long off = 0;
        if (lane == 0) off = atomicAdd(ra.head, (unsigned long long)cnt);
        const uint32_t olo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)off);
        const uint32_t ohi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(off >> 32));
        off = ((unsigned long long)ohi << 32) | olo;
        if (off + cnt > ra.cap) {
            status = HALF_RUNS_OVERFLOW;
        } else {
            // the run chain holds runs [j * RC, ...) in its j-th chunk, last chunk first
            wave_sync();
            int64_t j = ((int64_t)cnt + RC - 1) / RC - 1;
            for (int c = rcur; c >= 0 && j >= 0; j--) {
                const uint64_t lo = (uint64_t)j * RC;
                const uint32_t m = (uint32_t)min((uint64_t)RC, (uint64_t)cnt - lo);
                const uint32_t *src = (const uint32_t *)(chunk_ptr(pool, c) + 16);
                for (uint32_t q = lane; q < m; q += 64) ra.base[off + lo + q] = src[q];
                const int pc = (int)chunk_hdr(pool, c, 0);
                pool_free(pool, c, lane);
                c = pc;
            }
            rcur = -1;
            run_off = off;
            nruns = cnt;
        }
    }
    free_chain(pool, rcur, lane);
    free_chain(pool, cur, lane);
    return status;
}

template <int C, bool PERM, bool PERSIST>
__global__ void __launch_bounds__(64) k_ydrop_fused(const HalfTask *__restrict__ tasks, WorkQueue wq, SeqSetView T,
                                                    SeqSetView Qp, SeqSetView Qm, ScoreDesc sc, ChunkPool pool,
                                                    RunArena ra, HalfResult *__restrict__ res, int kcap) {
    static_assert(C <= 8, "one 32-bit record word per lane");
    static_assert(64 * C + 64 + RING_CHUNK <= RING, "target ring too small for the window");
    typedef Scorer<PERM> S;
    __shared__ int sub[40];
    __shared__ int prof[2][8];
    __shared__ uint8_t aring[RING], bring[RING];
    __shared__ uint2 tb_idx[TB_IDX];
    const int lane = threadIdx.x;
    if (lane < 40) sub[lane] = (lane & 7) < 5 ? sc.sub[lane >> 3][lane & 7] : 0;
    if (lane < 5) {
        uint32_t lo = 0;
        for (int b = 0; b < 4; b++) lo |= ((uint32_t)sc.sub[lane][b] & 0xffu) << (8 * b);
        prof[0][lane] = (int)lo;
        prof[1][lane] = (int)((uint32_t)sc.sub[lane][4] & 0xffu);
    }
    __syncthreads();
    const int e = sc.gap_extend, oe = sc.gap_open + sc.gap_extend, Y = sc.ydrop;

    int hint = (int)((blockIdx.x * 37u) % (unsigned)pool.nwords);
    const uint32_t CH = 1u << pool.shift;
    auto chunk = [&](int c) { return chunk_ptr(pool, c); };

    int64_t item = PERSIST ? -1 : (int64_t)blockIdx.x;
    const int64_t nq = wq.n_dev ? *wq.n_dev : wq.n;     // halves in the queue
    for (;;) {
        if (PERSIST) {
            unsigned int q = 0;
            if (lane == 0) q = atomicAdd(wq.head, 1u);
            q = (unsigned int)__builtin_amdgcn_readfirstlane((int)q);
            if ((int64_t)q >= nq) break;
            item = q;
        } else if (item >= nq) {
            break;      // a launch sized for more halves than the queue holds
        }
        const int64_t tid = wq.ids ? wq.ids[item] : item;
        const HalfTask tk = tasks[tid];
        const SeqSetView Q = tk.qset ? Qm : Qp;
        const int64_t nA = tk.nA, nB = tk.nB;
        const int64_t kmax = nA + nB;
        // 32-bit copies: the band never reaches ROW_LIMIT antidiagonals (the half stops there)
        const int nA32 = (int)min(nA, (int64_t)ROW_LIMIT + 4096);
        const int nB32 = (int)min(nB, (int64_t)ROW_LIMIT + 4096);
        const int kmax32 = (int)min(kmax, (int64_t)ROW_LIMIT + 4096);
        __syncthreads();
        int a_hi = 0, b_hi = 0;
        while (a_hi < 64 * C + 64) { ring_fill(aring, T, tk.a0, tk.adir, nA, a_hi, lane); a_hi += RING_CHUNK; }
        while (b_hi < 128) { ring_fill(bring, Q, tk.b0, tk.bdir, nB, b_hi, lane); b_hi += RING_CHUNK; }
        auto acode = [&](int ia) { return ia < 0 ? 4 : (int)aring[ia & (RING - 1)]; };
        auto bcode = [&](int jb) {
            if (jb < 0) return 4;
            if (jb < b_hi - RING) return codeB(Q, tk, jb);
            return (int)bring[jb & (RING - 1)];
        };
        auto plo_of = [&](int a) { return PERM ? prof[0][a] : a * 8; };
        auto phi_of = [&](int a) { return PERM ? prof[1][a] : 0; };
        // query codes of positions bw0 + lane (bwa) and bw0 + 64 + lane (bwb): the code
        // entering the band each antidiagonal is a register read, not an LDS round trip
        int bw0 = -(1 << 30), bwa = 4, bwb = 4;
        auto bcode_next = [&](int pos) {
            if (pos < bw0 || pos >= bw0 + 128) {
                while (b_hi < pos + 128) { ring_fill(bring, Q, tk.b0, tk.bdir, nB, b_hi, lane); b_hi += RING_CHUNK; }
                bw0 = pos - 64;
                bwa = bcode(bw0 + lane);
                bwb = bcode(bw0 + 64 + lane);
            }
            const int d = pos - bw0;
            return __builtin_amdgcn_readlane(d < 64 ? bwa : bwb, d & 63);
        };

        int H1[C], H2[C], E1[C], F1[C], Plo[C], Phi[C], Bs[C];
        int base = 0;
#pragma unroll
        for (int r = 0; r < C; r++) {
            const int i = lane * C + r;
            H1[r] = (i == 0) ? 0 : NEG;
            H2[r] = NEG;
            E1[r] = NEG;
            F1[r] = NEG;
            const int a = acode(i - 1);
            Plo[r] = plo_of(a);
            Phi[r] = phi_of(a);
            Bs[r] = S::bsel(i == 0 ? bcode(0) : 4);
        }
        int best = 0, bi = 0, bj = 0;
        uint64_t cells = 1;
        int lmin1 = 0, lmax1 = 0, lmin2 = 1, lmax2 = 0;
        // current chunk of the code chain: index, address, first antidiagonal, bytes used
        int cur = pool_alloc(pool, hint, lane);
        uint8_t *cb = nullptr;
        int k0 = 1;
        uint32_t fill = 16;
        int status = HALF_OK;
        if (cur < 0) {
            status = HALF_ARENA_OVERFLOW;
        } else {
            cb = chunk(cur);
            if (lane == 0) {
                ((uint32_t *)cb)[0] = 0xffffffffu;
                ((uint32_t *)cb)[1] = 1u;
            }
        }
        int k = 1;
        const int klong = kcap > 0 ? kcap : 0x7fffffff;
        const int kend = min(kmax32, min(klong, ROW_LIMIT - 1));
        for (; status == HALF_OK && k <= kend; k++) {
            int lo = 0x7fffffff, hi = -1;
            if (lmin1 <= lmax1) { lo = lmin1; hi = lmax1 + 1; }
            if (lmin2 <= lmax2) { lo = min(lo, lmin2 + 1); hi = max(hi, lmax2 + 1); }
            const int clo = max(0, k - nB32);
            const int chi = min(nA32, k);
            lo = max(lo, clo);
            hi = min(hi, chi);
            const bool nonempty = lo <= hi;
            {
                const int s = nonempty ? (lo - 1 - base) / C : 0;
                if (s >= 1) {
                    while (a_hi < base + (s + 64) * C + 64) {
                        ring_fill(aring, T, tk.a0, tk.adir, nA, a_hi, lane);
                        a_hi += RING_CHUNK;
                    }
                    if (s == 1) {
#pragma unroll
                        for (int r = 0; r < C; r++) {
                            const int i_new = base + 64 * C + r;
                            const int a = acode(i_new - 1);
                            const int fb = S::bsel(bcode(k - i_new - 1));
                            H1[r] = dpp_shl1(NEG, H1[r]);
                            H2[r] = dpp_shl1(NEG, H2[r]);
                            E1[r] = dpp_shl1(NEG, E1[r]);
                            F1[r] = dpp_shl1(NEG, F1[r]);
                            Plo[r] = dpp_shl1(plo_of(a), Plo[r]);
                            Phi[r] = dpp_shl1(phi_of(a), Phi[r]);
                            Bs[r] = dpp_shl1(fb, Bs[r]);
                        }
                    } else {
                        const int sl_ = min(s, 64);
                        const int src = (lane + sl_) & 63;
                        const bool from_next = lane + sl_ >= 64;
#pragma unroll
                        for (int r = 0; r < C; r++) {
                            const int i_new = base + s * C + lane * C + r;
                            const int h1 = __shfl(H1[r], src, 64), h2 = __shfl(H2[r], src, 64);
                            const int e1 = __shfl(E1[r], src, 64), f1 = __shfl(F1[r], src, 64);
                            const int pl = __shfl(Plo[r], src, 64), ph = __shfl(Phi[r], src, 64);
                            const int bs = __shfl(Bs[r], src, 64);
                            const int a = acode(i_new - 1);
                            H1[r] = from_next ? NEG : h1;
                            H2[r] = from_next ? NEG : h2;
                            E1[r] = from_next ? NEG : e1;
                            F1[r] = from_next ? NEG : f1;
                            Plo[r] = from_next ? plo_of(a) : pl;
                            Phi[r] = from_next ? phi_of(a) : ph;
                            Bs[r] = from_next ? S::bsel(bcode(k - i_new - 1)) : bs;
                        }
                    }
                    base += s * C;
                }
                if (nonempty && hi > base + 64 * C - 1) { status = HALF_WIDTH_OVERFLOW; break; }
            }
            const int thr = best - Y;
            const int upH = dpp_shr1(NEG, H1[C - 1]);
            const int upF = dpp_shr1(NEG, F1[C - 1]);
            const int upD = dpp_shr1(NEG, H2[C - 1]);
            int Hn[C], En[C], Fn[C];
            uint32_t nib = 0, lmask = 0;      // traceback codes, live rows of this lane (bit r)
            int lmax = NEG;
            auto cell_pass = [&](auto edge_tag) {
                constexpr bool EDGE = decltype(edge_tag)::value;
                const int i0 = base + lane * C;
#pragma unroll
                for (int r = 0; r < C; r++) {
                    const int Hu = r ? H1[r - 1] : upH;
                    const int Fu = r ? F1[r - 1] : upF;
                    const int Hd = r ? H2[r - 1] : upD;
                    const int hlo = H1[r] - oe, ele = E1[r] - e;
                    const int huo = Hu - oe, fue = Fu - e;
                    const int E = imax3(hlo, ele, NEG);
                    const int F = imax3(huo, fue, NEG);
                    const int G = Hd + S::score(Plo[r], Phi[r], Bs[r], sub);
                    const int H = imax3(G, E, F);
                    bool live = H >= thr;
                    if (EDGE) {
                        const bool v = (unsigned)(i0 + r - clo) <= (unsigned)(chi - clo);
                        live = live && v;
                        En[r] = v ? E : NEG;
                        Fn[r] = v ? F : NEG;
                    } else {
                        En[r] = E;
                        Fn[r] = F;
                    }
                    Hn[r] = live ? H : NEG;
                    lmask |= live ? (1u << r) : 0u;
                    const uint32_t code = (H == G ? 0u : (H == E ? 1u : 2u)) | (hlo >= ele ? 4u : 0u) |
                                          (huo >= fue ? 8u : 0u);
                    nib |= code << (4 * r);
                    lmax = imax(lmax, Hn[r]);
                }
            };
            const bool edge = base < clo || base + 64 * C - 1 > nA32;
            if (edge) cell_pass(std::true_type());
            else cell_pass(std::false_type());
            // live rows of the antidiagonal: first and last lane with a live row, then
            // that lane's first / last live row
            int lmin0, lmax0;
            {
                // branch-free: with no live row m is 0 and the selects give the empty range
                const uint64_t m = __ballot(lmask != 0);
                const int L1 = __builtin_ctzll(m | (1ull << 63)), L2 = 63 - __builtin_clzll(m | 1ull);
                const uint32_t f1 = (uint32_t)__builtin_amdgcn_readlane((int)lmask, L1);
                const uint32_t f2 = (uint32_t)__builtin_amdgcn_readlane((int)lmask, L2);
                lmin0 = m ? base + L1 * C + __builtin_ctz(f1 | 0x80000000u) : 1;
                lmax0 = m ? base + L2 * C + (31 - __builtin_clz(f2 | 1u)) : 0;
            }
            // record of antidiagonal k: rows of the lanes covering [lo, hi]
            {
                int l_lo = 0, l_hi = -1;
                if (nonempty) {
                    l_lo = (lo - base) / C;
                    l_hi = (hi - base) / C;
                }
                const uint32_t ng = (uint32_t)(l_hi - l_lo + 1);
                const uint32_t need = 4 * ng;
                if (fill + need + 8u * (uint32_t)(k - k0 + 1) > CH) {
                    const int nc = pool_alloc(pool, hint, lane);
                    if (nc < 0) { status = HALF_ARENA_OVERFLOW; break; }
                    if (lane == 0) {
                        ((uint32_t *)cb)[2] = fill;
                        uint32_t *nh = (uint32_t *)chunk(nc);
                        nh[0] = (uint32_t)cur;
                        nh[1] = (uint32_t)k;
                    }
                    cur = nc;
                    cb = chunk(nc);
                    k0 = k;
                    fill = 16;
                }
                // unconditional stores: lanes outside the record write the chunk header's
                // spare word, and every lane writes the same index entry
                uint32_t *rec = (uint32_t *)(cb + fill);
                const bool mine = lane >= l_lo && lane <= l_hi;
                *(mine ? rec + (lane - l_lo) : (uint32_t *)(cb + 12)) = nib;
                *(uint2 *)(cb + CH - 8u * (uint32_t)(k - k0 + 1)) =
                    make_uint2(fill, nonempty ? (uint32_t)(base + l_lo * C) : 0u);
                fill += need;
                cells += nonempty ? (uint64_t)(hi - lo + 1) : 0u;
            }
            // best: only when some live cell beats it; then the first row reaching the new maximum
            if (__ballot(lmax > best)) {
                const int admax = wave_max_dpp(lmax);
                uint32_t eq = 0;
#pragma unroll
                for (int r = 0; r < C; r++) eq |= (Hn[r] == admax) ? (1u << r) : 0u;
                const uint64_t m = __ballot(eq != 0);
                const int L = __builtin_ctzll(m);
                const int row = L * C + __builtin_ctz((uint32_t)__builtin_amdgcn_readlane((int)eq, L));
                best = admax;
                bi = base + row;
                bj = k - bi;
                if (best >= SFE_SCORE_LIMIT) { status = HALF_SCORE_RANGE; break; }
            }
#pragma unroll
            for (int r = 0; r < C; r++) {
                H2[r] = H1[r];
                H1[r] = Hn[r];
                E1[r] = En[r];
                F1[r] = Fn[r];
            }
            {
                const int carry = dpp_shr1(S::bsel(bcode_next(k - base)), Bs[C - 1]);
#pragma unroll
                for (int r = C - 1; r > 0; r--) Bs[r] = Bs[r - 1];
                Bs[0] = carry;
            }
            const bool stop = (lmin0 > lmax0) && (lmin1 > lmax1);
            lmin2 = lmin1; lmax2 = lmax1;
            lmin1 = lmin0; lmax1 = lmax0;
            if (stop) break;
        }

        if (status == HALF_OK && k > kend && k <= kmax32) status = k >= ROW_LIMIT ? HALF_SCORE_RANGE : HALF_LONG;
        if (cur >= 0 && lane == 0) ((uint32_t *)cb)[2] = fill;

        uint64_t run_off = 0;
        uint32_t nruns = 0;
        if (status == HALF_OK && (bi != 0 || bj != 0))
            status = trace_half<false>(pool, hint, lane, cur, bi, bj, C, ra, tb_idx, run_off, nruns);
        else
            free_chain(pool, cur, lane);
        if (lane == 0) {
            HalfResult o;
            o.best = best;
            o.i_end = bi;
            o.j_end = bj;
            o.status = status;
            o.cells = cells;
            o.tb_page = run_off;
            o.tb_end = nruns;
            o.k_last = (int32_t)min((int64_t)k, kmax);
            res[tid] = o;
        }
        if (!PERSIST) break;
    }
}

// ---------------------------------------------------------------------------
// The same extension in packed 16-bit arithmetic, two rows per register.
//
// Every value of antidiagonal k is held relative to that antidiagonal's
// Y-drop threshold t_k = (best over earlier antidiagonals) - Y, so a cell is
// live exactly when its value is >= 0; dead values saturate towards -32768
// (the 16-bit NEG).  When the best improves by d on antidiagonal k,
// t_{k+1} = t_k + d, and the operands read from antidiagonals k and k - 1 are
// lowered by the matching sums of improvements (folded into the gap
// penalties and the score bias).  Live values stay in [0, Y + max score], so
// the kernel is exact whenever Y + gap open + gap extend + twice the largest
// score magnitude stays well below 2^15 (checked by the host).  Ties and the
// traceback decisions are those of the 32-bit kernel: each decision compares
// two values of which the winner is live, and saturating subtraction keeps
// the sign of every difference.
//
// A lane's C rows form P = C / 2 pairs (p, p + P), row p in the low half of
// register p, so the row above pair p is pair p - 1 (pair 0: the lane above's
// last row and the lane's own row P - 1).  Substitution scores come from
// per-row profiles of biased bytes (score + 128) through v_perm, straight into
// the right half; two perms and one 32-bit add3 give both rows' diagonal
// candidates (a low half of at most 0x8000 + 255 never carries).
typedef short pk_i16 __attribute__((ext_vector_type(2)));
typedef unsigned short pk_u16 __attribute__((ext_vector_type(2)));
#define NEG2 ((int)0x80008000)

__device__ __forceinline__ int pk_subs(int a, int b) {
    return __builtin_bit_cast(int, __builtin_elementwise_sub_sat(__builtin_bit_cast(pk_i16, a), __builtin_bit_cast(pk_i16, b)));
}
__device__ __forceinline__ int pk_max(int a, int b) {
    return __builtin_bit_cast(int, __builtin_elementwise_max(__builtin_bit_cast(pk_i16, a), __builtin_bit_cast(pk_i16, b)));
}
// live (>= 0) values unchanged, negative values to -32768
__device__ __forceinline__ int pk_kill(int a) {
    return __builtin_bit_cast(int, __builtin_elementwise_min(__builtin_bit_cast(pk_u16, a), (pk_u16){0x8000, 0x8000}));
}
__device__ __forceinline__ uint32_t bfi(uint32_t m, uint32_t a, uint32_t b) { return (m & a) | (~m & b); }
__device__ __forceinline__ int pk2(int v) { return (int)(((uint32_t)v & 0xffffu) * 0x10001u); }
__device__ __forceinline__ int lo16(int v) { return (int)(short)(v & 0xffff); }
__device__ __forceinline__ int hi16(int v) { return v >> 16; }
// query-code selectors: the score byte lands in byte 0 (rows p) or byte 2 (rows p + P)
__device__ __forceinline__ int sel_lo(int code) { return 0x0c0c0c00 | code; }
__device__ __forceinline__ int sel_hi(int code) { return 0x0c000c0c | (code << 16); }
__device__ __forceinline__ int lo_of_hi(int x) { return (int)__builtin_amdgcn_perm((uint32_t)x, 0x0c0c0c0cu, 0x00000006u); }
__device__ __forceinline__ int hi_of_lo(int x) { return (int)__builtin_amdgcn_perm((uint32_t)x, 0x0c0c0c0cu, 0x00040000u); }

template <int C, bool PERSIST>
__global__ void __launch_bounds__(64) k_ydrop_fused16(const HalfTask *__restrict__ tasks, WorkQueue wq, SeqSetView T,
                                                      SeqSetView Qp, SeqSetView Qm, ScoreDesc sc, ChunkPool pool,
                                                      RunArena ra, HalfResult *__restrict__ res, int kcap) {
    static_assert(C % 2 == 0 && C <= 8, "rows in pairs, one 32-bit record word per lane");
    static_assert(64 * C + 64 + RING_CHUNK <= RING, "target ring too small for the window");
    constexpr int P = C / 2;
    __shared__ int prof[2][8];
    __shared__ uint8_t aring[RING], bring[RING];
    __shared__ uint2 tb_idx[TB_IDX];
    const int lane = threadIdx.x;
    if (lane < 5) {
        uint32_t lo = 0;
        for (int b = 0; b < 4; b++) lo |= ((uint32_t)(sc.sub[lane][b] + 128) & 0xffu) << (8 * b);
        prof[0][lane] = (int)lo;
        prof[1][lane] = (int)((uint32_t)(sc.sub[lane][4] + 128) & 0xffu);
    }
    __syncthreads();
    const int e = sc.gap_extend, oe = sc.gap_open + sc.gap_extend, Y = sc.ydrop;

    int hint = (int)((blockIdx.x * 37u) % (unsigned)pool.nwords);
    const uint32_t CH = 1u << pool.shift;
    auto chunk = [&](int c) { return chunk_ptr(pool, c); };

    int64_t item = PERSIST ? -1 : (int64_t)blockIdx.x;
    const int64_t nq = wq.n_dev ? *wq.n_dev : wq.n;     // halves in the queue
    for (;;) {
        if (PERSIST) {
            unsigned int q = 0;
            if (lane == 0) q = atomicAdd(wq.head, 1u);
            q = (unsigned int)__builtin_amdgcn_readfirstlane((int)q);
            if ((int64_t)q >= nq) break;
            item = q;
        } else if (item >= nq) {
            break;      // a launch sized for more halves than the queue holds
        }
        const int64_t tid = wq.ids ? wq.ids[item] : item;
        const HalfTask tk = tasks[tid];
        const SeqSetView Q = tk.qset ? Qm : Qp;
        const int64_t nA = tk.nA, nB = tk.nB;
        const int64_t kmax = nA + nB;
        const int nA32 = (int)min(nA, (int64_t)ROW_LIMIT + 4096);
        const int nB32 = (int)min(nB, (int64_t)ROW_LIMIT + 4096);
        const int kmax32 = (int)min(kmax, (int64_t)ROW_LIMIT + 4096);
        __syncthreads();
        int a_hi = 0, b_hi = 0;
        while (a_hi < 64 * C + 64) { ring_fill(aring, T, tk.a0, tk.adir, nA, a_hi, lane); a_hi += RING_CHUNK; }
        while (b_hi < 128) { ring_fill(bring, Q, tk.b0, tk.bdir, nB, b_hi, lane); b_hi += RING_CHUNK; }
        auto acode = [&](int ia) { return ia < 0 ? 4 : (int)aring[ia & (RING - 1)]; };
        auto bcode = [&](int jb) {
            if (jb < 0) return 4;
            if (jb < b_hi - RING) return codeB(Q, tk, jb);
            return (int)bring[jb & (RING - 1)];
        };
        int bw0 = -(1 << 30), bwa = 4, bwb = 4;
        auto bcode_next = [&](int pos) {
            if (pos < bw0 || pos >= bw0 + 128) {
                while (b_hi < pos + 128) { ring_fill(bring, Q, tk.b0, tk.bdir, nB, b_hi, lane); b_hi += RING_CHUNK; }
                bw0 = pos - 64;
                bwa = bcode(bw0 + lane);
                bwb = bcode(bw0 + 64 + lane);
            }
            const int d = pos - bw0;
            return __builtin_amdgcn_readlane(d < 64 ? bwa : bwb, d & 63);
        };
        auto sel_row = [&](int r, int code) { return r < P ? sel_lo(code) : sel_hi(code); };

        // pairs: H1/E1/F1 antidiagonal k - 1 (relative to t_{k-1}), H2 antidiagonal k - 2 (t_{k-2})
        int H1[P], H2[P], E1[P], F1[P];
        int Plo[C], Phi[C], Bs[C];
        int base = 0;
#pragma unroll
        for (int p = 0; p < P; p++) {
            H1[p] = (lane == 0 && p == 0) ? (int)(0x80000000u | (uint32_t)Y) : NEG2;   // cell (0, 0): 0 - t_0 = Y
            H2[p] = NEG2;
            E1[p] = NEG2;
            F1[p] = NEG2;
        }
#pragma unroll
        for (int r = 0; r < C; r++) {
            const int i = lane * C + r;
            const int a = acode(i - 1);
            Plo[r] = prof[0][a];
            Phi[r] = prof[1][a];
            Bs[r] = sel_row(r, i == 0 ? bcode(0) : 4);
        }
        int best = 0, bi = 0, bj = 0;
        int d1 = 0, d2 = 0;               // t_k - t_{k-1}, t_{k-1} - t_{k-2}
        uint64_t cells = 1;
        int lmin1 = 0, lmax1 = 0, lmin2 = 1, lmax2 = 0;
        int cur = pool_alloc(pool, hint, lane);
        uint8_t *cb = nullptr;
        int k0 = 1;
        uint32_t fill = 16;
        int status = HALF_OK;
        if (cur < 0) {
            status = HALF_ARENA_OVERFLOW;
        } else {
            cb = chunk(cur);
            if (lane == 0) {
                ((uint32_t *)cb)[0] = 0xffffffffu;
                ((uint32_t *)cb)[1] = 1u;
            }
        }
        int k = 1;
        const int klong = kcap > 0 ? kcap : 0x7fffffff;
        const int kend = min(kmax32, min(klong, ROW_LIMIT - 1));
        for (; status == HALF_OK && k <= kend; k++) {
            int lo = 0x7fffffff, hi = -1;
            if (lmin1 <= lmax1) { lo = lmin1; hi = lmax1 + 1; }
            if (lmin2 <= lmax2) { lo = min(lo, lmin2 + 1); hi = max(hi, lmax2 + 1); }
            const int clo = max(0, k - nB32);
            const int chi = min(nA32, k);
            lo = max(lo, clo);
            hi = min(hi, chi);
            const bool nonempty = lo <= hi;
            {
                const int s = nonempty ? (lo - 1 - base) / C : 0;
                if (s >= 1) {
                    while (a_hi < base + (s + 64) * C + 64) {
                        ring_fill(aring, T, tk.a0, tk.adir, nA, a_hi, lane);
                        a_hi += RING_CHUNK;
                    }
                    if (s == 1) {
#pragma unroll
                        for (int p = 0; p < P; p++) {
                            H1[p] = dpp_shl1(NEG2, H1[p]);
                            H2[p] = dpp_shl1(NEG2, H2[p]);
                            E1[p] = dpp_shl1(NEG2, E1[p]);
                            F1[p] = dpp_shl1(NEG2, F1[p]);
                        }
#pragma unroll
                        for (int r = 0; r < C; r++) {
                            const int i_new = base + 64 * C + r;
                            const int a = acode(i_new - 1);
                            Plo[r] = dpp_shl1(prof[0][a], Plo[r]);
                            Phi[r] = dpp_shl1(prof[1][a], Phi[r]);
                            Bs[r] = dpp_shl1(sel_row(r, bcode(k - i_new - 1)), Bs[r]);
                        }
                    } else {
                        const int sl_ = min(s, 64);
                        const int src = (lane + sl_) & 63;
                        const bool from_next = lane + sl_ >= 64;
#pragma unroll
                        for (int p = 0; p < P; p++) {
                            const int h1 = __shfl(H1[p], src, 64), h2 = __shfl(H2[p], src, 64);
                            const int e1 = __shfl(E1[p], src, 64), f1 = __shfl(F1[p], src, 64);
                            H1[p] = from_next ? NEG2 : h1;
                            H2[p] = from_next ? NEG2 : h2;
                            E1[p] = from_next ? NEG2 : e1;
                            F1[p] = from_next ? NEG2 : f1;
                        }
#pragma unroll
                        for (int r = 0; r < C; r++) {
                            const int i_new = base + s * C + lane * C + r;
                            const int pl = __shfl(Plo[r], src, 64), ph = __shfl(Phi[r], src, 64);
                            const int bs = __shfl(Bs[r], src, 64);
                            const int a = acode(i_new - 1);
                            Plo[r] = from_next ? prof[0][a] : pl;
                            Phi[r] = from_next ? prof[1][a] : ph;
                            Bs[r] = from_next ? sel_row(r, bcode(k - i_new - 1)) : bs;
                        }
                    }
                    base += s * C;
                }
                if (nonempty && hi > base + 64 * C - 1) { status = HALF_WIDTH_OVERFLOW; break; }
            }
            const int oeD = pk2(oe + d1), eD = pk2(e + d1), gD = pk2(128 + d1 + d2);
            const int upH = (int)__builtin_amdgcn_alignbit((uint32_t)H1[P - 1], (uint32_t)dpp_shr1(NEG2, H1[P - 1]), 16);
            const int upF = (int)__builtin_amdgcn_alignbit((uint32_t)F1[P - 1], (uint32_t)dpp_shr1(NEG2, F1[P - 1]), 16);
            const int upD = (int)__builtin_amdgcn_alignbit((uint32_t)H2[P - 1], (uint32_t)dpp_shr1(NEG2, H2[P - 1]), 16);
            int Hn[P], En[P], Fn[P];
            uint32_t nib = 0;
            auto cell_pass = [&](auto edge_tag) {
                constexpr bool EDGE = decltype(edge_tag)::value;
                const int i0 = base + lane * C;
#pragma unroll
                for (int p = 0; p < P; p++) {
                    const int Hu = p ? H1[p - 1] : upH;
                    const int Fu = p ? F1[p - 1] : upF;
                    const int Hd = p ? H2[p - 1] : upD;
                    const int hlo = pk_subs(H1[p], oeD), ele = pk_subs(E1[p], eD);
                    const int huo = pk_subs(Hu, oeD), fue = pk_subs(Fu, eD);
                    const int E = pk_max(hlo, ele), F = pk_max(huo, fue);
                    const int sE = pk_subs(hlo, ele), sF = pk_subs(huo, fue);
                    const uint32_t s2 = (uint32_t)Hd +
                                        __builtin_amdgcn_perm((uint32_t)Phi[p], (uint32_t)Plo[p], (uint32_t)Bs[p]) +
                                        __builtin_amdgcn_perm((uint32_t)Phi[p + P], (uint32_t)Plo[p + P], (uint32_t)Bs[p + P]);
                    const int G = pk_subs((int)s2, gD);
                    const int t = pk_max(E, F);
                    const int H = pk_max(G, t);
                    const int sD = pk_subs(G, t), sEF = pk_subs(E, F);
                    int h = pk_kill(H);
                    if (EDGE) {
                        const bool vl = (unsigned)(i0 + p - clo) <= (unsigned)(chi - clo);
                        const bool vh = (unsigned)(i0 + p + P - clo) <= (unsigned)(chi - clo);
                        const uint32_t m = (vl ? 0x0000ffffu : 0u) | (vh ? 0xffff0000u : 0u);
                        En[p] = (int)bfi(m, (uint32_t)E, (uint32_t)NEG2);
                        Fn[p] = (int)bfi(m, (uint32_t)F, (uint32_t)NEG2);
                        h = (int)bfi(m, (uint32_t)h, (uint32_t)NEG2);
                    } else {
                        En[p] = E;
                        Fn[p] = F;
                    }
                    Hn[p] = h;
                    const uint32_t ca = bfi(0x80008000u, (uint32_t)sD, (uint32_t)sEF >> 1);
                    const uint32_t cb2 = bfi(0x80008000u, (uint32_t)sE, (uint32_t)sF >> 1);
                    const uint32_t cc = bfi(0xC000C000u, ca, cb2 >> 2);
                    nib = p ? bfi(0xF000F000u >> (4 * p), cc >> (4 * p), nib) : cc;
                }
            };
            const bool edge = base < clo || base + 64 * C - 1 > nA32;
            if (edge) cell_pass(std::true_type());
            else cell_pass(std::false_type());
            // live rows: bit p (row p) and bit 16 + p (row p + P) of lmask
            uint32_t dead = 0;
#pragma unroll
            for (int p = 0; p < P; p++) dead |= ((uint32_t)Hn[p] >> (15 - p)) & (0x00010001u << p);
            // live rows of the lane in row order (bit r = row r)
            const uint32_t live = ~dead & (((1u << P) - 1u) * 0x10001u);
            const uint32_t lmask = (live & 0xffffu) | ((live >> 16) << P);
            int lmin0, lmax0;
            {
                // branch-free: with no live row m is 0 and the selects give the empty range
                const uint64_t m = __ballot(lmask != 0);
                const int L1 = __builtin_ctzll(m | (1ull << 63)), L2 = 63 - __builtin_clzll(m | 1ull);
                const uint32_t f1 = (uint32_t)__builtin_amdgcn_readlane((int)lmask, L1);
                const uint32_t f2 = (uint32_t)__builtin_amdgcn_readlane((int)lmask, L2);
                lmin0 = m ? base + L1 * C + __builtin_ctz(f1 | 0x80000000u) : 1;
                lmax0 = m ? base + L2 * C + (31 - __builtin_clz(f2 | 1u)) : 0;
            }
            {
                int l_lo = 0, l_hi = -1;
                if (nonempty) {
                    l_lo = (lo - base) / C;
                    l_hi = (hi - base) / C;
                }
                const uint32_t ng = (uint32_t)(l_hi - l_lo + 1);
                const uint32_t need = 4 * ng;
                if (fill + need + 8u * (uint32_t)(k - k0 + 1) > CH) {
                    const int nc = pool_alloc(pool, hint, lane);
                    if (nc < 0) { status = HALF_ARENA_OVERFLOW; break; }
                    if (lane == 0) {
                        ((uint32_t *)cb)[2] = fill;
                        uint32_t *nh = (uint32_t *)chunk(nc);
                        nh[0] = (uint32_t)cur;
                        nh[1] = (uint32_t)k;
                    }
                    cur = nc;
                    cb = chunk(nc);
                    k0 = k;
                    fill = 16;
                }
                // unconditional stores: lanes outside the record write the chunk header's
                // spare word, and every lane writes the same index entry
                uint32_t *rec = (uint32_t *)(cb + fill);
                const bool mine = lane >= l_lo && lane <= l_hi;
                *(mine ? rec + (lane - l_lo) : (uint32_t *)(cb + 12)) = nib;
                *(uint2 *)(cb + CH - 8u * (uint32_t)(k - k0 + 1)) =
                    make_uint2(fill, nonempty ? (uint32_t)(base + l_lo * C) : 0u);
                fill += need;
                cells += nonempty ? (uint64_t)(hi - lo + 1) : 0u;
            }
            // best: a live value above Y (relative to t_k) beats it; then the first row reaching the maximum
            int mx = Hn[0];
#pragma unroll
            for (int p = 1; p < P; p++) mx = pk_max(mx, Hn[p]);
            mx = imax(lo16(mx), hi16(mx));
            int dnow = 0;
            if (__ballot(mx > Y)) {
                const int admax = wave_max_dpp(mx);
                // every value is <= admax: a half equals it exactly when its difference is not negative
                const int a2 = pk2(admax);
                uint32_t below = 0;
#pragma unroll
                for (int p = 0; p < P; p++)
                    below |= ((uint32_t)pk_subs(Hn[p], a2) >> (15 - p)) & (0x00010001u << p);
                const uint32_t eqh = ~below & (((1u << P) - 1u) * 0x10001u);
                const uint32_t eq = (eqh & 0xffffu) | ((eqh >> 16) << P);
                const uint64_t m = __ballot(eq != 0);
                const int L = __builtin_ctzll(m);
                const uint32_t f = (uint32_t)__builtin_amdgcn_readlane((int)eq, L);
                const int row = L * C + __builtin_ctz(f);
                dnow = admax - Y;
                best += dnow;
                bi = base + row;
                bj = k - bi;
                if (best >= SFE_SCORE_LIMIT) { status = HALF_SCORE_RANGE; break; }
            }
            d2 = d1;
            d1 = dnow;
#pragma unroll
            for (int p = 0; p < P; p++) {
                H2[p] = H1[p];
                H1[p] = Hn[p];
                E1[p] = En[p];
                F1[p] = Fn[p];
            }
            {
                // rows move down by one: row 0 takes the lane above's row C - 1 (lane 0: the code entering)
                const int carry = lo_of_hi(dpp_shr1(sel_hi(bcode_next(k - base)), Bs[C - 1]));
                const int into_hi = hi_of_lo(Bs[P - 1]);
#pragma unroll
                for (int r = C - 1; r > 0; r--) Bs[r] = (r == P) ? into_hi : Bs[r - 1];
                Bs[0] = carry;
            }
            const bool stop = (lmin0 > lmax0) && (lmin1 > lmax1);
            lmin2 = lmin1; lmax2 = lmax1;
            lmin1 = lmin0; lmax1 = lmax0;
            if (stop) break;
        }

        if (status == HALF_OK && k > kend && k <= kmax32) status = k >= ROW_LIMIT ? HALF_SCORE_RANGE : HALF_LONG;
        if (cur >= 0 && lane == 0) ((uint32_t *)cb)[2] = fill;

        uint64_t run_off = 0;
        uint32_t nruns = 0;
        if (status == HALF_OK && (bi != 0 || bj != 0))
            status = trace_half<true>(pool, hint, lane, cur, bi, bj, C, ra, tb_idx, run_off, nruns);
        else
            free_chain(pool, cur, lane);
        if (lane == 0) {
            HalfResult o;
            o.best = best;
            o.i_end = bi;
            o.j_end = bj;
            o.status = status;
            o.cells = cells;
            o.tb_page = run_off;
            o.tb_end = nruns;
            o.k_last = (int32_t)min((int64_t)k, kmax);
            res[tid] = o;
        }
        if (!PERSIST) break;
    }
}
#undef NEG2

// ---------------------------------------------------------------------------
// Wave-group extension of one long half (Sec. 8: a long anchor-half spread over
// several warps instead of one).  W waves own consecutive slabs of the window
// (wave w: lanes w*64 .. w*64+63 of the group, C rows each).  Per antidiagonal
// each wave computes its slab; the row above its first row, the query code that
// crosses into it, its lane 0 (needed when the window slides by one lane) and
// its share of the reductions (live rows, best) go through LDS, and one
// barrier per antidiagonal makes them visible.  Every wave then derives the
// same uniform state (range, slide, best, chunk), so control flow never
// diverges across the barrier.  The records have the single-wave format with
// W*64 lane groups; wave 0 traces the half back afterwards.
template <int C, int W>
struct CoopXch {
    int bnd[4];           // lane 63, row C-1 after the update: H, F, H of k-1, query code before the shift
    int l0[7 * C];        // lane 0 after the update: H1, H2, E1, F1, Plo, Phi, Bs (Bs[0] placeholder)
    int lmin, lmax;       // live rows of the wave (lmin > lmax: none)
    int vmax, vrow;       // wave maximum of live H and its first row (when above the best)
    int newchunk, pad;    // wave 0: chunk for the next antidiagonal (-1 none, -2 pool dry)
};

template <int C, int W, bool PERM>
__global__ void __launch_bounds__(64 * W) k_ydrop_coop(const HalfTask *__restrict__ tasks,
                                                       const int32_t *__restrict__ ids, SeqSetView T, SeqSetView Qp,
                                                       SeqSetView Qm, ScoreDesc sc, ChunkPool pool, RunArena ra,
                                                       HalfResult *__restrict__ res) {
    static_assert(C <= 8, "one 32-bit record word per lane");
    typedef Scorer<PERM> S;
    constexpr int NT = 64 * W;            // lanes of the group
    constexpr int NR = NT * C;            // rows of the window
    constexpr int NV = 7 * C;             // registers of one lane
    // target codes of the whole window plus margin and a refill chunk
    constexpr int ARING = NR + 64 + RING_CHUNK <= RING ? RING : (NR + 64 + RING_CHUNK <= 2048 ? 2048 : 4096);
    static_assert(NR + 64 + RING_CHUNK <= ARING, "target ring too small for the window");
    __shared__ int sub[40];
    __shared__ int prof[2][8];
    __shared__ uint8_t aring[ARING], bring[RING];
    __shared__ uint2 tb_idx[TB_IDX];
    __shared__ CoopXch<C, W> xch[2][W];
    __shared__ int dump[NT * NV];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    if (tid < 40) sub[tid] = (tid & 7) < 5 ? sc.sub[tid >> 3][tid & 7] : 0;
    if (tid < 5) {
        uint32_t lo = 0;
        for (int b = 0; b < 4; b++) lo |= ((uint32_t)sc.sub[tid][b] & 0xffu) << (8 * b);
        prof[0][tid] = (int)lo;
        prof[1][tid] = (int)((uint32_t)sc.sub[tid][4] & 0xffu);
    }
    __syncthreads();
    const int e = sc.gap_extend, oe = sc.gap_open + sc.gap_extend, Y = sc.ydrop;
    int hint = (int)((blockIdx.x * 37u) % (unsigned)pool.nwords);
    const uint32_t CH = 1u << pool.shift;
    const int64_t hid = ids ? ids[blockIdx.x] : (int64_t)blockIdx.x;
    const HalfTask tk = tasks[hid];
    const SeqSetView Q = tk.qset ? Qm : Qp;
    const int64_t nA = tk.nA, nB = tk.nB;
    const int64_t kmax = nA + nB;
    const int nA32 = (int)min(nA, (int64_t)ROW_LIMIT + 4096);
    const int nB32 = (int)min(nB, (int64_t)ROW_LIMIT + 4096);
    const int kmax32 = (int)min(kmax, (int64_t)ROW_LIMIT + 4096);
    int a_hi = 0, b_hi = 0;
    while (a_hi < NR + 64) { ring_fill<NT, ARING>(aring, T, tk.a0, tk.adir, nA, a_hi, tid); a_hi += RING_CHUNK; }
    while (b_hi < 128) { ring_fill<NT>(bring, Q, tk.b0, tk.bdir, nB, b_hi, tid); b_hi += RING_CHUNK; }
    auto acode = [&](int ia) { return ia < 0 ? 4 : (int)aring[ia & (ARING - 1)]; };
    auto bcode = [&](int jb) {
        if (jb < 0) return 4;
        if (jb < b_hi - RING) return codeB(Q, tk, jb);
        return (int)bring[jb & (RING - 1)];
    };
    auto plo_of = [&](int a) { return PERM ? prof[0][a] : a * 8; };
    auto phi_of = [&](int a) { return PERM ? prof[1][a] : 0; };
    int bw0 = -(1 << 30), bwa = 4, bwb = 4;
    auto bcode_next = [&](int pos) {          // uniform position; every wave calls it
        if (pos < bw0 || pos >= bw0 + 128) {
            while (b_hi < pos + 128) { ring_fill<NT>(bring, Q, tk.b0, tk.bdir, nB, b_hi, tid); b_hi += RING_CHUNK; }
            bw0 = pos - 64;
            bwa = bcode(bw0 + lane);
            bwb = bcode(bw0 + 64 + lane);
        }
        const int d = pos - bw0;
        return d < 64 ? __builtin_amdgcn_readlane(bwa, d) : __builtin_amdgcn_readlane(bwb, d - 64);
    };

    int H1[C], H2[C], E1[C], F1[C], Plo[C], Phi[C], Bs[C];
    int base = 0;
#pragma unroll
    for (int r = 0; r < C; r++) {
        const int i = tid * C + r;
        H1[r] = (i == 0) ? 0 : NEG;
        H2[r] = NEG;
        E1[r] = NEG;
        F1[r] = NEG;
        const int a = acode(i - 1);
        Plo[r] = plo_of(a);
        Phi[r] = phi_of(a);
        Bs[r] = S::bsel(i == 0 ? bcode(0) : 4);
    }
    int best = 0, bi = 0, bj = 0;
    uint64_t cells = 1;
    int lmin1 = 0, lmax1 = 0, lmin2 = 1, lmax2 = 0;
    int status = HALF_OK;
    // chunk of the code chain (uniform): wave 0 takes it, everyone learns it through LDS
    if (w == 0) {
        const int c0 = pool_alloc(pool, hint, lane);
        if (lane == 0) {
            xch[1][0].newchunk = c0 >= 0 ? c0 : -2;
            if (c0 >= 0) {
                ((uint32_t *)chunk_ptr(pool, c0))[0] = 0xffffffffu;
                ((uint32_t *)chunk_ptr(pool, c0))[1] = 1u;
            }
        }
    }
    __syncthreads();
    int cur = xch[1][0].newchunk;
    if (cur < 0) { status = HALF_ARENA_OVERFLOW; cur = -1; }
    uint8_t *cb = cur >= 0 ? chunk_ptr(pool, cur) : nullptr;
    int k0 = 1;
    uint32_t fill = 16;
    constexpr uint32_t MAXNEED = 4 * NT;
    int k = 1;
    for (; status == HALF_OK && k <= kmax32; k++) {
        if (k >= ROW_LIMIT) { status = HALF_SCORE_RANGE; break; }
        const int par = k & 1, prv = par ^ 1;
        // the query code that crossed from wave w-1 into this wave's lane 0
        if (k >= 2 && w > 0 && lane == 0) Bs[0] = xch[prv][w - 1].bnd[3];
        int lo = 0x7fffffff, hi = -1;
        if (lmin1 <= lmax1) { lo = lmin1; hi = lmax1 + 1; }
        if (lmin2 <= lmax2) { lo = min(lo, lmin2 + 1); hi = max(hi, lmax2 + 1); }
        const int clo = max(0, k - nB32);
        const int chi = min(nA32, k);
        lo = max(lo, clo);
        hi = min(hi, chi);
        const bool nonempty = lo <= hi;
        // the row above this wave's first row (wave 0: none)
        int bH = NEG, bF = NEG, bD = NEG;
        if (w > 0 && k >= 2) {
            bH = xch[prv][w - 1].bnd[0];
            bF = xch[prv][w - 1].bnd[1];
            bD = xch[prv][w - 1].bnd[2];
        }
        if (nonempty) {
            const int s = (lo - 1 - base) / C;
            if (s >= 1) {
                while (a_hi < base + s * C + NR + 64) {
                    ring_fill<NT, ARING>(aring, T, tk.a0, tk.adir, nA, a_hi, tid);
                    a_hi += RING_CHUNK;
                }
                if (s == 1 && k >= 2) {
                    // lane 63 takes the next wave's lane 0 (the last wave: new rows)
#pragma unroll
                    for (int r = 0; r < C; r++) {
                        int iH1, iH2, iE1, iF1, iPlo, iPhi, iBs;
                        if (w < W - 1) {
                            const int *l0 = xch[prv][w + 1].l0;
                            iH1 = l0[r];
                            iH2 = l0[C + r];
                            iE1 = l0[2 * C + r];
                            iF1 = l0[3 * C + r];
                            iPlo = l0[4 * C + r];
                            iPhi = l0[5 * C + r];
                            iBs = r ? l0[6 * C + r] : xch[prv][w].bnd[3];
                        } else {
                            const int i_new = base + NR + r;
                            const int a = acode(i_new - 1);
                            iH1 = iH2 = iE1 = iF1 = NEG;
                            iPlo = plo_of(a);
                            iPhi = phi_of(a);
                            iBs = S::bsel(bcode(k - i_new - 1));
                        }
                        H1[r] = dpp_shl1(iH1, H1[r]);
                        H2[r] = dpp_shl1(iH2, H2[r]);
                        E1[r] = dpp_shl1(iE1, E1[r]);
                        F1[r] = dpp_shl1(iF1, F1[r]);
                        Plo[r] = dpp_shl1(iPlo, Plo[r]);
                        Phi[r] = dpp_shl1(iPhi, Phi[r]);
                        Bs[r] = dpp_shl1(iBs, Bs[r]);
                    }
                    // the row above wave w's new first row was wave w's old lane 0, row C-1
                    if (w > 0) {
                        const int *l0 = xch[prv][w].l0;
                        bH = l0[C - 1];
                        bF = l0[3 * C + C - 1];
                        bD = l0[C + C - 1];
                    }
                } else {
                    // any shift: through the whole window in LDS
#pragma unroll
                    for (int r = 0; r < C; r++) {
                        int *d = dump + tid * NV;
                        d[r] = H1[r];
                        d[C + r] = H2[r];
                        d[2 * C + r] = E1[r];
                        d[3 * C + r] = F1[r];
                        d[4 * C + r] = Plo[r];
                        d[5 * C + r] = Phi[r];
                        d[6 * C + r] = Bs[r];
                    }
                    __syncthreads();
                    const int src = tid + s;
#pragma unroll
                    for (int r = 0; r < C; r++) {
                        if (src < NT) {
                            const int *d = dump + src * NV;
                            H1[r] = d[r];
                            H2[r] = d[C + r];
                            E1[r] = d[2 * C + r];
                            F1[r] = d[3 * C + r];
                            Plo[r] = d[4 * C + r];
                            Phi[r] = d[5 * C + r];
                            Bs[r] = d[6 * C + r];
                        } else {
                            const int i_new = base + s * C + tid * C + r;
                            const int a = acode(i_new - 1);
                            H1[r] = H2[r] = E1[r] = F1[r] = NEG;
                            Plo[r] = plo_of(a);
                            Phi[r] = phi_of(a);
                            Bs[r] = S::bsel(bcode(k - i_new - 1));
                        }
                    }
                    bH = bF = bD = NEG;
                    const int up = w * 64 - 1 + s;          // old lane of the row above wave w's first row
                    if (w > 0 && up < NT) {
                        const int *d = dump + up * NV;
                        bH = d[C - 1];
                        bF = d[3 * C + C - 1];
                        bD = d[C + C - 1];
                    }
                    __syncthreads();
                }
                base += s * C;
            }
            if (hi > base + NR - 1) { status = HALF_WIDTH_OVERFLOW; break; }
        }
        const int thr = best - Y;
        const int upH = dpp_shr1(bH, H1[C - 1]);
        const int upF = dpp_shr1(bF, F1[C - 1]);
        const int upD = dpp_shr1(bD, H2[C - 1]);
        int Hn[C], En[C], Fn[C];
        uint32_t nib = 0, lmask = 0;
        int lmax = NEG;
        auto cell_pass = [&](auto edge_tag) {
            constexpr bool EDGE = decltype(edge_tag)::value;
            const int i0 = base + tid * C;
#pragma unroll
            for (int r = 0; r < C; r++) {
                const int Hu = r ? H1[r - 1] : upH;
                const int Fu = r ? F1[r - 1] : upF;
                const int Hd = r ? H2[r - 1] : upD;
                const int hlo = H1[r] - oe, ele = E1[r] - e;
                const int huo = Hu - oe, fue = Fu - e;
                const int E = imax3(hlo, ele, NEG);
                const int F = imax3(huo, fue, NEG);
                const int G = Hd + S::score(Plo[r], Phi[r], Bs[r], sub);
                const int H = imax3(G, E, F);
                bool live = H >= thr;
                if (EDGE) {
                    const bool v = (unsigned)(i0 + r - clo) <= (unsigned)(chi - clo);
                    live = live && v;
                    En[r] = v ? E : NEG;
                    Fn[r] = v ? F : NEG;
                } else {
                    En[r] = E;
                    Fn[r] = F;
                }
                Hn[r] = live ? H : NEG;
                lmask |= live ? (1u << r) : 0u;
                const uint32_t code = (H == G ? 0u : (H == E ? 1u : 2u)) | (hlo >= ele ? 4u : 0u) |
                                      (huo >= fue ? 8u : 0u);
                nib |= code << (4 * r);
                lmax = imax(lmax, Hn[r]);
            }
        };
        const bool edge = base < clo || base + NR - 1 > nA32;
        if (edge) cell_pass(std::true_type());
        else cell_pass(std::false_type());
        // this wave's share of the reductions
        int wmin = 1, wmax = 0;
        {
            const uint64_t m = __ballot(lmask != 0);
            if (m) {
                const int L1 = __builtin_ctzll(m), L2 = 63 - __builtin_clzll(m);
                const uint32_t f1 = (uint32_t)__builtin_amdgcn_readlane((int)lmask, L1);
                const uint32_t f2 = (uint32_t)__builtin_amdgcn_readlane((int)lmask, L2);
                wmin = base + (w * 64 + L1) * C + __builtin_ctz(f1);
                wmax = base + (w * 64 + L2) * C + (31 - __builtin_clz(f2));
            }
        }
        int vmax = NEG, vrow = 0x7fffffff;
        if (__ballot(lmax > best)) {
            vmax = wave_max_dpp(lmax);
            uint32_t eq = 0;
#pragma unroll
            for (int r = 0; r < C; r++) eq |= (Hn[r] == vmax) ? (1u << r) : 0u;
            const uint64_t m = __ballot(eq != 0);
            const int L = __builtin_ctzll(m);
            vrow = base + (w * 64 + L) * C + __builtin_ctz((uint32_t)__builtin_amdgcn_readlane((int)eq, L));
        }
        // record of antidiagonal k: the lane groups covering [lo, hi]
        int g_lo = 0, g_hi = -1;
        if (nonempty) {
            g_lo = (lo - base) / C;
            g_hi = (hi - base) / C;
        }
        const uint32_t ng = (uint32_t)(g_hi - g_lo + 1);
        const uint32_t need = 4 * ng;
        {
            uint32_t *rec = (uint32_t *)(cb + fill);
            if (tid >= g_lo && tid <= g_hi) rec[tid - g_lo] = nib;
            if (tid == 0)
                *(uint2 *)(cb + CH - 8u * (uint32_t)(k - k0 + 1)) =
                    make_uint2(fill, nonempty ? (uint32_t)(base + g_lo * C) : 0u);
        }
        fill += need;
        if (nonempty) cells += (uint64_t)(hi - lo + 1);
        // state update and the query-code shift (the code entering wave 0)
        const int bs_out = Bs[C - 1];
        const int code_in = S::bsel(bcode_next(k - base));
        {
            const int carry = dpp_shr1(w == 0 ? code_in : S::bsel(4), Bs[C - 1]);
#pragma unroll
            for (int r = C - 1; r > 0; r--) Bs[r] = Bs[r - 1];
            Bs[0] = carry;
        }
        CoopXch<C, W> &X = xch[par][w];
        if (lane == 63) {
            X.bnd[0] = Hn[C - 1];
            X.bnd[1] = Fn[C - 1];
            X.bnd[2] = H1[C - 1];
            X.bnd[3] = bs_out;
        }
#pragma unroll
        for (int r = 0; r < C; r++) {
            H2[r] = H1[r];
            H1[r] = Hn[r];
            E1[r] = En[r];
            F1[r] = Fn[r];
        }
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < C; r++) {
                X.l0[r] = H1[r];
                X.l0[C + r] = H2[r];
                X.l0[2 * C + r] = E1[r];
                X.l0[3 * C + r] = F1[r];
                X.l0[4 * C + r] = Plo[r];
                X.l0[5 * C + r] = Phi[r];
                X.l0[6 * C + r] = Bs[r];
            }
            X.lmin = wmin;
            X.lmax = wmax;
            X.vmax = vmax;
            X.vrow = vrow;
        }
        // room for the next antidiagonal's record: wave 0 takes a new chunk now
        if (w == 0) {
            int nc = -1;
            if (fill + MAXNEED + 8u * (uint32_t)(k + 1 - k0 + 1) > CH) {
                nc = pool_alloc(pool, hint, lane);
                if (nc >= 0 && lane == 0) {
                    ((uint32_t *)cb)[2] = fill;
                    uint32_t *nh = (uint32_t *)chunk_ptr(pool, nc);
                    nh[0] = (uint32_t)cur;
                    nh[1] = (uint32_t)(k + 1);
                }
                if (nc < 0) nc = -2;
            }
            if (lane == 0) X.newchunk = nc;
        }
        __syncthreads();
        // uniform state from every wave's share
        int lmin0 = 1, lmax0 = 0, gmax = NEG, grow = 0x7fffffff;
#pragma unroll
        for (int v = 0; v < W; v++) {
            const CoopXch<C, W> &Z = xch[par][v];
            if (Z.lmin <= Z.lmax) {
                if (lmin0 > lmax0) { lmin0 = Z.lmin; lmax0 = Z.lmax; }
                else { lmin0 = min(lmin0, Z.lmin); lmax0 = max(lmax0, Z.lmax); }
            }
            if (Z.vmax > gmax) { gmax = Z.vmax; grow = Z.vrow; }
        }
        if (gmax > best) {
            best = gmax;
            bi = grow;
            bj = k - bi;
            if (best >= SFE_SCORE_LIMIT) { status = HALF_SCORE_RANGE; break; }
        }
        const int nc = xch[par][0].newchunk;
        if (nc == -2) { status = HALF_ARENA_OVERFLOW; break; }
        if (nc >= 0) {
            cur = nc;
            cb = chunk_ptr(pool, nc);
            k0 = k + 1;
            fill = 16;
        }
        const bool stop = (lmin0 > lmax0) && (lmin1 > lmax1);
        lmin2 = lmin1; lmax2 = lmax1;
        lmin1 = lmin0; lmax1 = lmax0;
        if (stop) break;
    }
    __syncthreads();
    if (cur >= 0 && tid == 0) ((uint32_t *)cb)[2] = fill;
    __syncthreads();
    if (w == 0) {
        uint64_t run_off = 0;
        uint32_t nruns = 0;
        if (status == HALF_OK && (bi != 0 || bj != 0))
            status = trace_half<false>(pool, hint, lane, cur, bi, bj, C, ra, tb_idx, run_off, nruns);
        else
            free_chain(pool, cur, lane);
        if (lane == 0) {
            HalfResult o;
            o.best = best;
            o.i_end = bi;
            o.j_end = bj;
            o.status = status;
            o.cells = cells;
            o.tb_page = run_off;
            o.tb_end = nruns;
            o.k_last = (int32_t)min((int64_t)k, kmax);
            res[hid] = o;
        }
    }
}

void launch_ydrop_coop(int cells_per_lane, bool perm, const HalfTask *tasks, const int32_t *ids, int64_t n,
                       SeqSetView T, SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc, ChunkPool pool, RunArena ra,
                       HalfResult *res, hipStream_t st) {
    if (n <= 0) return;
    if (cells_per_lane <= 2) {
        if (perm) k_ydrop_coop<2, 4, true><<<(unsigned)n, 256, 0, st>>>(tasks, ids, T, Qp, Qm, sc, pool, ra, res);
        else k_ydrop_coop<2, 4, false><<<(unsigned)n, 256, 0, st>>>(tasks, ids, T, Qp, Qm, sc, pool, ra, res);
    } else {
        if (perm) k_ydrop_coop<4, 4, true><<<(unsigned)n, 256, 0, st>>>(tasks, ids, T, Qp, Qm, sc, pool, ra, res);
        else k_ydrop_coop<4, 4, false><<<(unsigned)n, 256, 0, st>>>(tasks, ids, T, Qp, Qm, sc, pool, ra, res);
    }
}

void launch_ydrop_fused(int cells_per_lane, bool perm, bool narrow, bool persistent, const HalfTask *tasks,
                        WorkQueue wq, int64_t grid, SeqSetView T, SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc,
                        ChunkPool pool, RunArena ra, HalfResult *res, int kcap, size_t dyn_lds, hipStream_t st) {
    if (grid <= 0) return;
    if (narrow) {
#define SFE_LAUNCH16(CC, QQ) \
    k_ydrop_fused16<CC, QQ><<<(unsigned)grid, 64, dyn_lds, st>>>(tasks, wq, T, Qp, Qm, sc, pool, ra, res, kcap)
#define SFE_BY_C16(QQ)                                    \
    do {                                                  \
        if (cells_per_lane <= 2) SFE_LAUNCH16(2, QQ);     \
        else if (cells_per_lane <= 4) SFE_LAUNCH16(4, QQ); \
        else if (cells_per_lane <= 6) SFE_LAUNCH16(6, QQ); \
        else SFE_LAUNCH16(8, QQ);                         \
    } while (0)
        if (persistent) SFE_BY_C16(true); else SFE_BY_C16(false);
#undef SFE_BY_C16
#undef SFE_LAUNCH16
        return;
    }
#define SFE_LAUNCH(CC, PP, QQ) \
    k_ydrop_fused<CC, PP, QQ><<<(unsigned)grid, 64, dyn_lds, st>>>(tasks, wq, T, Qp, Qm, sc, pool, ra, res, kcap)
#define SFE_BY_C(PP, QQ)                                  \
    do {                                                  \
        if (cells_per_lane <= 2) SFE_LAUNCH(2, PP, QQ);   \
        else if (cells_per_lane <= 3) SFE_LAUNCH(3, PP, QQ); \
        else if (cells_per_lane <= 4) SFE_LAUNCH(4, PP, QQ); \
        else if (cells_per_lane <= 6) SFE_LAUNCH(6, PP, QQ); \
        else SFE_LAUNCH(8, PP, QQ);                       \
    } while (0)
    if (perm) {
        if (persistent) SFE_BY_C(true, true); else SFE_BY_C(true, false);
    } else {
        if (persistent) SFE_BY_C(false, true); else SFE_BY_C(false, false);
    }
#undef SFE_BY_C
#undef SFE_LAUNCH
}

int ydrop_fused_blocks_per_cu(int cells_per_lane, bool perm, bool narrow, bool persistent, size_t dyn_lds) {
    int nb = 0;
    hipError_t err = hipSuccess;
    if (narrow) {
#define SFE_OCC16(CC, QQ) err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ydrop_fused16<CC, QQ>, 64, dyn_lds)
#define SFE_OCC_C16(QQ)                                   \
    do {                                                  \
        if (cells_per_lane <= 2) SFE_OCC16(2, QQ);        \
        else if (cells_per_lane <= 4) SFE_OCC16(4, QQ);   \
        else if (cells_per_lane <= 6) SFE_OCC16(6, QQ);   \
        else SFE_OCC16(8, QQ);                            \
    } while (0)
        if (persistent) SFE_OCC_C16(true); else SFE_OCC_C16(false);
#undef SFE_OCC_C16
#undef SFE_OCC16
        return err == hipSuccess ? nb : -1;
    }
#define SFE_OCC(CC, PP, QQ) err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ydrop_fused<CC, PP, QQ>, 64, dyn_lds)
#define SFE_OCC_C(PP, QQ)                                 \
    do {                                                  \
        if (cells_per_lane <= 2) SFE_OCC(2, PP, QQ);      \
        else if (cells_per_lane <= 3) SFE_OCC(3, PP, QQ); \
        else if (cells_per_lane <= 4) SFE_OCC(4, PP, QQ); \
        else if (cells_per_lane <= 6) SFE_OCC(6, PP, QQ); \
        else SFE_OCC(8, PP, QQ);                          \
    } while (0)
    if (perm) {
        if (persistent) SFE_OCC_C(true, true); else SFE_OCC_C(true, false);
    } else {
        if (persistent) SFE_OCC_C(false, true); else SFE_OCC_C(false, false);
    }
#undef SFE_OCC_C
#undef SFE_OCC
    return err == hipSuccess ? nb : -1;
}

}  // namespace sfe
