// k_extend.hip -- gapped Y-drop extension of anchor halves on gfx950
// (Sec. 8 of the paper), traceback and assembly of alignments.
//
// The DP of a half (A = target side, B = query side, both read away from the
// anchor column):
//   H(0,0) = 0, E(0,0) = F(0,0) = NEG
//   E(i,j) = max(H(i,j-1) - (o+e), E(i,j-1) - e)     gap consuming B (op I)
//   F(i,j) = max(H(i-1,j) - (o+e), F(i-1,j) - e)     gap consuming A (op D)
//   G(i,j) = H(i-1,j-1) + sub[A(i-1)][B(j-1)]
//   H(i,j) = max(G, E, F)
// evaluated antidiagonal by antidiagonal (k = i + j).  A cell is live when
// H >= best_{k-1} - Y, best_{k-1} being the best live H on antidiagonals
// before k (0 before the first); reading a cell that is not live (or was
// never computed) gives NEG.  Antidiagonal k computes rows
//   [min(minrow(live k-1), minrow(live k-2) + 1), max(maxrow(live k-1), maxrow(live k-2)) + 1]
// clipped to the matrix; the half stops after two antidiagonals without a
// live cell.  Its end is the first live cell (smallest k, then smallest row)
// reaching the final best.
//
// Wavefront mapping (the systolic idea of Sec. 8, re-thought for 64-wide
// waves): one wave owns a window of 64*C consecutive rows, C rows per lane
// (lane l holds rows base + l*C .. base + l*C + C-1).  The three values a
// cell needs from row i-1 (H and F of antidiagonal k-1, H of k-2) come from
// the same lane or, for the lane's first row, from the previous lane by a
// cross-lane shift; the query base of a cell moves one row down per
// antidiagonal, so the query codes travel through the lanes as a shift
// register fed by one new code per antidiagonal.  The window slides forward
// (whole lanes at a time) as the band of live rows moves along the diagonal.
// A band wider than the window is reported and the half is re-run with a
// wider window, or by the workgroup kernel, which has no width limit.
//
// Dead cells keep their E and F values (instead of NEG) in the wave kernel:
// such values are below the current threshold, the threshold never
// decreases, and every path through them stays below it, so no live value
// and no pointer on a traceback path depends on them.
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

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = imax(v, __shfl_xor(v, m, 64));
    return v;
}

// Half tasks of the batch items: task 2x is the forward half, 2x+1 the backward half.
__global__ void k_make_tasks(const ExtItem *__restrict__ items, int64_t n, const UnitDesc *__restrict__ units,
                             int64_t nt, HalfTask *__restrict__ tasks) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    ExtItem it = items[x];
    UnitDesc u = units[it.unit];
    HalfTask f, b;
    f.a0 = (int64_t)it.ta + 1; f.adir = 1; f.nA = nt - it.ta - 1;
    f.b0 = u.seq_start + it.qa + 1; f.bdir = 1; f.nB = u.len - it.qa - 1;
    f.qset = u.strand; f.pad = 0;
    b.a0 = (int64_t)it.ta - 1; b.adir = -1; b.nA = it.ta;
    b.b0 = u.seq_start + (int64_t)it.qa - 1; b.bdir = -1; b.nB = it.qa;
    b.qset = u.strand; b.pad = 0;
    tasks[2 * x] = f;
    tasks[2 * x + 1] = b;
}

void launch_make_tasks(const ExtItem *items, int64_t n, const UnitDesc *units, int64_t nt, HalfTask *tasks,
                       hipStream_t st) {
    if (n <= 0) return;
    k_make_tasks<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(items, n, units, nt, tasks);
}

// ---------------------------------------------------------------------------
// Arena: page allocation and record writing (uniform across the wave or done
// by one thread of a workgroup)
// ---------------------------------------------------------------------------
struct PageCursor {
    uint64_t page;      // arena offset of the current allocation, ~0 if none
    uint32_t fill;      // bytes used in it
    uint32_t size;      // bytes in it
};

// Makes room for `need` bytes; returns false when the arena is exhausted.
// Called by one thread (the caller broadcasts the cursor).
__device__ __forceinline__ bool arena_reserve_1t(Arena &ar, PageCursor &pc, uint32_t need) {
    if (pc.page != ~0ull && pc.fill + need <= pc.size) return true;
    uint32_t pages = (need + ARENA_HDR + ARENA_PAGE - 1) / ARENA_PAGE;
    unsigned long long off = atomicAdd(ar.head, (unsigned long long)pages * ARENA_PAGE);
    if (off + (unsigned long long)pages * ARENA_PAGE > ar.bytes) return false;
    uint32_t *hdr = (uint32_t *)(ar.base + off);
    uint64_t prev = pc.page;
    hdr[0] = (uint32_t)prev;
    hdr[1] = (uint32_t)(prev >> 32);
    hdr[2] = pc.fill;
    hdr[3] = pages;
    pc.page = off;
    pc.fill = ARENA_HDR;
    pc.size = pages * ARENA_PAGE;
    return true;
}

// ---------------------------------------------------------------------------
// Wave kernel
// ---------------------------------------------------------------------------
template <int C>
__global__ void __launch_bounds__(64) k_ydrop_wave(const HalfTask *__restrict__ tasks, const int32_t *__restrict__ ids,
                                                   SeqSetView T, SeqSetView Qp, SeqSetView Qm, ScoreDesc sc,
                                                   Arena ar, HalfResult *__restrict__ res) {
    __shared__ int sub[40];
    const int lane = threadIdx.x;
    if (lane < 40) sub[lane] = (lane & 7) < 5 ? sc.sub[lane >> 3][lane & 7] : 0;
    __syncthreads();
    const int64_t tid = ids ? ids[blockIdx.x] : blockIdx.x;
    const HalfTask tk = tasks[tid];
    const SeqSetView Q = tk.qset ? Qm : Qp;
    const int e = sc.gap_extend, oe = sc.gap_open + sc.gap_extend, Y = sc.ydrop;
    const int64_t nA = tk.nA, nB = tk.nB;

    int H1[C], H2[C], E1[C], F1[C], A8[C], Bc[C];
    int64_t base = 0;
#pragma unroll
    for (int r = 0; r < C; r++) {
        int64_t i = (int64_t)lane * C + r;
        H1[r] = (i == 0) ? 0 : NEG;
        H2[r] = NEG;
        E1[r] = NEG;
        F1[r] = NEG;
        A8[r] = (i >= 1 ? codeA(T, tk, i - 1) : 4) * 8;
        Bc[r] = codeB(Q, tk, 1 - i - 1);
    }
    int best = 0;
    int64_t bi = 0, bj = 0;
    uint64_t cells = 1;
    int64_t lmin1 = 0, lmax1 = 0;           // live rows of antidiagonal k-1 (lmin > lmax: none)
    int64_t lmin2 = 1, lmax2 = 0;           // live rows of antidiagonal k-2
    PageCursor pc;
    pc.page = ~0ull; pc.fill = 0; pc.size = 0;
    uint64_t tb_page = ~0ull;
    uint32_t tb_end = 0;
    int status = HALF_OK;
    int64_t k = 1;
    const int64_t kmax = nA + nB;
    for (; k <= kmax; k++) {
        // candidate rows of antidiagonal k
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        if (lmin1 <= lmax1) { lo = lmin1; hi = lmax1 + 1; }
        if (lmin2 <= lmax2) { lo = min(lo, lmin2 + 1); hi = max(hi, lmax2 + 1); }
        const int64_t clo = max((int64_t)0, k - nB), chi = min(nA, k);
        bool nonempty = false;
        if (lo != INT64_MAX) {
            lo = max(lo, clo);
            hi = min(hi, chi);
            nonempty = lo <= hi;
        }
        if (nonempty) {
            // slide the window: rows below lo-1 are never read again
            int64_t s = (lo - 1 - base) / C;
            if (s > 0) {
                const int sl = (int)min(s, (int64_t)64);
#pragma unroll
                for (int r = 0; r < C; r++) {
                    H1[r] = __shfl(H1[r], lane + sl, 64);
                    H2[r] = __shfl(H2[r], lane + sl, 64);
                    E1[r] = __shfl(E1[r], lane + sl, 64);
                    F1[r] = __shfl(F1[r], lane + sl, 64);
                    A8[r] = __shfl(A8[r], lane + sl, 64);
                    Bc[r] = __shfl(Bc[r], lane + sl, 64);
                }
                base += s * C;
                if (lane + sl >= 64) {
#pragma unroll
                    for (int r = 0; r < C; r++) {
                        int64_t i = base + (int64_t)lane * C + r;
                        H1[r] = NEG; H2[r] = NEG; E1[r] = NEG; F1[r] = NEG;
                        A8[r] = codeA(T, tk, i - 1) * 8;
                        Bc[r] = codeB(Q, tk, k - i - 1);
                    }
                }
            }
            if (hi > base + 64 * C - 1) { status = HALF_WIDTH_OVERFLOW; break; }
        }
        const int thr = best - Y;
        // values of row i-1 for each lane's first row
        int upH = __shfl_up(H1[C - 1], 1, 64);
        int upF = __shfl_up(F1[C - 1], 1, 64);
        int upD = __shfl_up(H2[C - 1], 1, 64);
        if (lane == 0) { upH = NEG; upF = NEG; upD = NEG; }
        int Hn[C], En[C], Fn[C];
        typedef typename std::conditional<(C > 8), uint64_t, uint32_t>::type NibT;   // 4 bits per row
        NibT nib = 0;
        int lmax = NEG;
        int64_t larg = 0, lfirst = INT64_MAX, llast = -1;
#pragma unroll
        for (int r = 0; r < C; r++) {
            const int64_t i = base + (int64_t)lane * C + r;
            const int Hu = r ? H1[r - 1] : upH;
            const int Fu = r ? F1[r - 1] : upF;
            const int Hd = r ? H2[r - 1] : upD;
            const int hlo = H1[r] - oe, ele = E1[r] - e;
            const int huo = Hu - oe, fue = Fu - e;
            const int E = imax3(hlo, ele, NEG);
            const int F = imax3(huo, fue, NEG);
            const int G = Hd + sub[A8[r] + Bc[r]];
            const int H = imax3(G, E, F);
            const bool v = i >= clo && i <= chi;
            const bool live = v && H >= thr;
            Hn[r] = live ? H : NEG;
            En[r] = v ? E : NEG;
            Fn[r] = v ? F : NEG;
            NibT code = (H == G ? 0u : (H == E ? 1u : 2u)) | (hlo >= ele ? 4u : 0u) | (huo >= fue ? 8u : 0u);
            nib |= code << (4 * r);
            if (live) {
                if (H > lmax) { lmax = H; larg = i; }
                if (lfirst == INT64_MAX) lfirst = i;
                llast = i;
            }
        }
        // live rows of this antidiagonal
        const uint64_t anylive = __ballot(llast >= 0);
        int64_t lmin0 = 1, lmax0 = 0;
        if (anylive) {
            int fl = __ffsll((unsigned long long)anylive) - 1;
            int ll = 63 - __clzll((unsigned long long)anylive);
            lmin0 = __shfl(lfirst, fl, 64);
            lmax0 = __shfl(llast, ll, 64);
        }
        // traceback record of this antidiagonal: rows of the lanes covering [lo, hi]
        {
            int64_t l_lo = 0, l_hi = -1;
            if (nonempty) {
                l_lo = (lo - base) / C;
                l_hi = (hi - base) / C;
            }
            const uint32_t n = (uint32_t)((l_hi - l_lo + 1) * C);
            const uint32_t pbytes = rec_payload_bytes(n);
            const uint32_t need = pbytes + 8;
            bool ok = true;
            if (lane == 0) ok = arena_reserve_1t(ar, pc, need);
            ok = __shfl(ok ? 1 : 0, 0, 64) != 0;
            pc.page = __shfl(pc.page, 0, 64);
            pc.fill = __shfl(pc.fill, 0, 64);
            pc.size = __shfl(pc.size, 0, 64);
            if (!ok) { status = HALF_ARENA_OVERFLOW; break; }
            uint8_t *rec = ar.base + pc.page + pc.fill;
            if (lane >= l_lo && lane <= l_hi) {
                uint8_t *dst = rec + (lane - l_lo) * (C / 2);
                if (C == 4) {
                    *(uint16_t *)dst = (uint16_t)nib;
                } else {
#pragma unroll
                    for (int b = 0; b < C / 2; b++) dst[b] = (uint8_t)(nib >> (8 * b));
                }
            }
            if (lane == 0) {
                uint32_t *ft = (uint32_t *)(rec + pbytes);
                ft[0] = (uint32_t)(nonempty ? base + l_lo * C : 0);
                ft[1] = n;
            }
            pc.fill += need;
            if (nonempty) cells += (uint64_t)(hi - lo + 1);
        }
        // best over this antidiagonal; end cell = smallest row reaching it
        const int admax = wave_max(lmax);
        if (admax > best) {
            const uint64_t m = __ballot(lmax == admax);
            const int fl = __ffsll((unsigned long long)m) - 1;
            const int64_t row = __shfl(larg, fl, 64);
            best = admax;
            bi = row;
            bj = k - row;
            tb_page = pc.page;
            tb_end = pc.fill;
        }
        // advance
#pragma unroll
        for (int r = 0; r < C; r++) {
            H2[r] = H1[r];
            H1[r] = Hn[r];
            E1[r] = En[r];
            F1[r] = Fn[r];
        }
        const int64_t bnew = k - base;       // B index of row `base` on antidiagonal k+1
        int carry = __shfl_up(Bc[C - 1], 1, 64);
#pragma unroll
        for (int r = C - 1; r > 0; r--) Bc[r] = Bc[r - 1];
        Bc[0] = lane == 0 ? codeB(Q, tk, bnew) : carry;
        const bool stop = (lmin0 > lmax0) && (lmin1 > lmax1);
        lmin2 = lmin1; lmax2 = lmax1;
        lmin1 = lmin0; lmax1 = lmax0;
        if (stop) break;
    }
    if (lane == 0) {
        HalfResult o;
        o.best = best;
        o.i_end = (int32_t)bi;
        o.j_end = (int32_t)bj;
        o.status = status;
        o.cells = cells;
        o.tb_page = tb_page;
        o.tb_end = tb_end;
        o.k_last = (int32_t)min(k, kmax);
        res[tid] = o;
    }
}

void launch_ydrop(int cells_per_lane, const HalfTask *tasks, const int32_t *ids, int64_t n, SeqSetView T,
                  SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc, Arena arena, HalfResult *res, hipStream_t st) {
    if (n <= 0) return;
    if (cells_per_lane <= 4)
        k_ydrop_wave<4><<<(unsigned)n, 64, 0, st>>>(tasks, ids, T, Qp, Qm, sc, arena, res);
    else
        k_ydrop_wave<16><<<(unsigned)n, 64, 0, st>>>(tasks, ids, T, Qp, Qm, sc, arena, res);
}

// ---------------------------------------------------------------------------
// Workgroup kernel without a width limit: one workgroup of 256 threads per
// half, the last two antidiagonals in ring buffers of cap rows (global
// memory), dead cells stored as NEG.  Used for halves whose band outgrows the
// wave kernel's window; reports HALF_WIDTH_OVERFLOW if the band outgrows cap.
// ---------------------------------------------------------------------------
#define RING_T 256
__global__ void __launch_bounds__(RING_T) k_ydrop_ring(const HalfTask *__restrict__ tasks, const int32_t *__restrict__ ids,
                                                       SeqSetView T, SeqSetView Qp, SeqSetView Qm, ScoreDesc sc,
                                                       Arena ar, int32_t *__restrict__ ring, int32_t cap,
                                                       HalfResult *__restrict__ res) {
    __shared__ int sub[40];
    __shared__ unsigned long long s_best;      // (H + 2^31) << 32 | ~row : max = best H, smallest row
    __shared__ long long s_min, s_max;
    __shared__ PageCursor s_pc;
    __shared__ int s_ok;
    const int t = threadIdx.x;
    if (t < 40) sub[t] = (t & 7) < 5 ? sc.sub[t >> 3][t & 7] : 0;
    const int64_t tid = ids ? ids[blockIdx.x] : blockIdx.x;
    const HalfTask tk = tasks[tid];
    const SeqSetView Q = tk.qset ? Qm : Qp;
    const int e = sc.gap_extend, oe = sc.gap_open + sc.gap_extend, Y = sc.ydrop;
    const int64_t nA = tk.nA, nB = tk.nB;
    const int64_t mask = cap - 1;
    // ring layout: H[3][cap], E[2][cap], F[2][cap]
    int32_t *Hr = ring + (int64_t)blockIdx.x * 7 * cap;
    int32_t *Er = Hr + 3 * (int64_t)cap;
    int32_t *Fr = Er + 2 * (int64_t)cap;
    if (t == 0) {
        Hr[0] = 0; Er[0] = NEG; Fr[0] = NEG;
        s_pc.page = ~0ull; s_pc.fill = 0; s_pc.size = 0;
    }
    __syncthreads();
    int best = 0;
    int64_t bi = 0, bj = 0;
    uint64_t cells = 1;
    int64_t lmin1 = 0, lmax1 = 0, lmin2 = 1, lmax2 = 0;
    int64_t lo1 = 0, hi1 = 0, lo2 = 1, hi2 = 0;      // computed rows of k-1, k-2
    uint64_t tb_page = ~0ull;
    uint32_t tb_end = 0;
    int status = HALF_OK;
    int64_t k = 1;
    const int64_t kmax = nA + nB;
    for (; k <= kmax; k++) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        if (lmin1 <= lmax1) { lo = lmin1; hi = lmax1 + 1; }
        if (lmin2 <= lmax2) { lo = min(lo, lmin2 + 1); hi = max(hi, lmax2 + 1); }
        bool nonempty = false;
        if (lo != INT64_MAX) {
            lo = max(lo, max((int64_t)0, k - nB));
            hi = min(hi, min(nA, k));
            nonempty = lo <= hi;
        }
        if (nonempty && hi - lo + 3 > cap) { status = HALF_WIDTH_OVERFLOW; break; }
        if (t == 0) { s_best = 0; s_min = INT64_MAX; s_max = -1; }
        const uint32_t n = nonempty ? (uint32_t)(hi - lo + 1) : 0u;
        const uint32_t pbytes = rec_payload_bytes(n);
        if (t == 0) s_ok = arena_reserve_1t(ar, s_pc, pbytes + 8) ? 1 : 0;
        __syncthreads();
        if (!s_ok) { status = HALF_ARENA_OVERFLOW; break; }
        uint8_t *rec = ar.base + s_pc.page + s_pc.fill;
        const int thr = best - Y;
        const int c1 = (int)((k - 1) % 3), c2 = (int)((k + 1) % 3), c0 = (int)(k % 3);  // k-1, k-2, k
        const int e1 = (int)((k - 1) & 1), e0 = (int)(k & 1);
        if (nonempty) {
            for (int64_t i0 = lo + 2 * (int64_t)t; i0 <= hi; i0 += 2 * RING_T) {
                uint32_t byte = 0;
                for (int u = 0; u < 2; u++) {
                    const int64_t i = i0 + u;
                    if (i > hi) break;
                    const int64_t j = k - i;
                    const bool in1 = i >= lo1 && i <= hi1, in1u = i - 1 >= lo1 && i - 1 <= hi1;
                    const bool in2 = i - 1 >= lo2 && i - 1 <= hi2;
                    const int Hl = in1 ? Hr[c1 * cap + (i & mask)] : NEG;
                    const int El = in1 ? Er[e1 * cap + (i & mask)] : NEG;
                    const int Hu = in1u ? Hr[c1 * cap + ((i - 1) & mask)] : NEG;
                    const int Fu = in1u ? Fr[e1 * cap + ((i - 1) & mask)] : NEG;
                    const int Hd = in2 ? Hr[c2 * cap + ((i - 1) & mask)] : NEG;
                    const int hlo = Hl - oe, ele = El - e, huo = Hu - oe, fue = Fu - e;
                    const int E = imax3(hlo, ele, NEG);
                    const int F = imax3(huo, fue, NEG);
                    int G = NEG;
                    if (i >= 1 && j >= 1) G = imax(Hd + sub[codeA(T, tk, i - 1) * 8 + codeB(Q, tk, j - 1)], NEG);
                    const int H = imax3(G, E, F);
                    const bool live = H >= thr;
                    Hr[c0 * cap + (i & mask)] = live ? H : NEG;
                    Er[e0 * cap + (i & mask)] = live ? E : NEG;
                    Fr[e0 * cap + (i & mask)] = live ? F : NEG;
                    uint32_t code = (H == G ? 0u : (H == E ? 1u : 2u)) | (hlo >= ele ? 4u : 0u) | (huo >= fue ? 8u : 0u);
                    byte |= code << (4 * u);
                    if (live) {
                        unsigned long long key = ((unsigned long long)(uint32_t)(H + 0x80000000u) << 32) |
                                                 (unsigned long long)(0xffffffffu - (uint32_t)i);
                        atomicMax(&s_best, key);
                        atomicMin(&s_min, (long long)i);
                        atomicMax(&s_max, (long long)i);
                    }
                }
                rec[(i0 - lo) >> 1] = (uint8_t)byte;
            }
        }
        __syncthreads();
        if (t == 0) {
            uint32_t *ft = (uint32_t *)(rec + pbytes);
            ft[0] = nonempty ? (uint32_t)lo : 0u;
            ft[1] = n;
            s_pc.fill += pbytes + 8;
        }
        __syncthreads();
        if (nonempty) cells += (uint64_t)(hi - lo + 1);
        int64_t lmin0 = 1, lmax0 = 0;
        if (s_max >= 0) { lmin0 = s_min; lmax0 = s_max; }
        if (s_best != 0) {
            const int adm = (int)((uint32_t)(s_best >> 32) - 0x80000000u);
            if (adm > best) {
                best = adm;
                bi = (int64_t)(0xffffffffu - (uint32_t)(s_best & 0xffffffffu));
                bj = k - bi;
                tb_page = s_pc.page;
                tb_end = s_pc.fill;
            }
        }
        const bool stop = (lmin0 > lmax0) && (lmin1 > lmax1);
        lmin2 = lmin1; lmax2 = lmax1; lmin1 = lmin0; lmax1 = lmax0;
        lo2 = lo1; hi2 = hi1;
        if (nonempty) { lo1 = lo; hi1 = hi; } else { lo1 = 1; hi1 = 0; }
        __syncthreads();
        if (stop) break;
    }
    if (t == 0) {
        HalfResult o;
        o.best = best;
        o.i_end = (int32_t)bi;
        o.j_end = (int32_t)bj;
        o.status = status;
        o.cells = cells;
        o.tb_page = tb_page;
        o.tb_end = tb_end;
        o.k_last = (int32_t)min(k, kmax);
        res[tid] = o;
    }
}

void launch_ydrop_ring(const HalfTask *tasks, const int32_t *ids, int64_t n, SeqSetView T, SeqSetView Qp,
                       SeqSetView Qm, const ScoreDesc &sc, Arena arena, int32_t *ring, int32_t cap_rows,
                       HalfResult *res, hipStream_t st) {
    if (n <= 0) return;
    k_ydrop_ring<<<(unsigned)n, RING_T, 0, st>>>(tasks, ids, T, Qp, Qm, sc, arena, ring, cap_rows, res);
}

// ---------------------------------------------------------------------------
// Assembly: score, box and cells of each item from its two halves.
// ---------------------------------------------------------------------------
__global__ void k_assemble(const ExtItem *__restrict__ items, int64_t n, const UnitDesc *__restrict__ units,
                           const HalfResult *__restrict__ res, SeqSetView T, SeqSetView Qp, SeqSetView Qm,
                           ScoreDesc sc, sfe_aln *__restrict__ out) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    ExtItem it = items[x];
    UnitDesc u = units[it.unit];
    HalfResult f = res[2 * x], b = res[2 * x + 1];
    int ca = base_code(T, it.ta);
    int cq = base_code(u.strand ? Qm : Qp, u.seq_start + it.qa);
    sfe_aln a;
    a.score = sc.sub[ca][cq] + f.best + b.best;
    a.t_start = it.ta - b.i_end;
    a.t_end = it.ta + 1 + f.i_end;
    a.q_start = it.qa - b.j_end;
    a.q_end = it.qa + 1 + f.j_end;
    a.query_id = (uint32_t)u.query_id;
    a.anchor_t = it.ta;
    a.anchor_q = it.qa;
    a.ops_offset = 0;
    a.cells = f.cells + b.cells;
    a.ops_len = 0;
    a.strand = (uint8_t)u.strand;
    a.flags = a.score >= sc.gapped_thresh ? SFE_ALN_PASSED : 0;
    a.pad[0] = a.pad[1] = 0;
    out[x] = a;
}

void launch_assemble(const ExtItem *items, int64_t n, const UnitDesc *units, const HalfResult *res,
                     SeqSetView T, SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc, sfe_aln *out,
                     hipStream_t st) {
    if (n <= 0) return;
    k_assemble<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(items, n, units, res, T, Qp, Qm, sc, out);
}

// ---------------------------------------------------------------------------
// Traceback: walk the pointer records back from the end cell.  In state H the
// code's source field picks diagonal / E / F; in E (F) the open bit decides
// whether the gap started here.  Runs are emitted end cell first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rec_footer(const uint8_t *base, uint64_t page, uint32_t end, uint32_t &r0, uint32_t &n) {
    const uint32_t *ft = (const uint32_t *)(base + page + end - 8);
    r0 = ft[0];
    n = ft[1];
}

__global__ void k_traceback(const HalfResult *__restrict__ res, const int32_t *__restrict__ half_ids, int64_t nh,
                            Arena ar, const uint64_t *__restrict__ run_off, uint32_t *__restrict__ runs,
                            uint32_t *__restrict__ nruns) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nh) return;
    const int32_t h = half_ids[x];
    const HalfResult R = res[h];
    uint32_t *out = runs + run_off[x];
    int64_t i = R.i_end, j = R.j_end;
    uint32_t cnt = 0;
    if (i == 0 && j == 0) { nruns[x] = 0; return; }
    uint64_t page = R.tb_page;
    uint32_t end = R.tb_end;
    int64_t k = i + j;             // antidiagonal of the record ending at (page, end)
    int state = 0;
    uint32_t cur_op = 0xffffffffu, cur_len = 0;
    const uint32_t cap = (uint32_t)(R.i_end + R.j_end + 1);
    int64_t guard = 2 * (i + j) + 4;
    bool bad = false;
    while (!(i == 0 && j == 0 && state == 0)) {
        if (--guard < 0 || i < 0 || j < 0) { bad = true; break; }
        while (k > i + j) {
            uint32_t r0, n;
            rec_footer(ar.base, page, end, r0, n);
            uint32_t pb = rec_payload_bytes(n);
            if (end < ARENA_HDR + 8 + pb) { bad = true; break; }
            uint32_t start = end - 8 - pb;
            if (start == ARENA_HDR) {
                const uint32_t *hdr = (const uint32_t *)(ar.base + page);
                page = (uint64_t)hdr[0] | ((uint64_t)hdr[1] << 32);
                end = hdr[2];
                if (page >= ar.bytes || end < ARENA_HDR + 8) { bad = true; break; }
            } else {
                end = start;
            }
            k--;
        }
        if (bad) break;
        uint32_t r0, n;
        rec_footer(ar.base, page, end, r0, n);
        const uint8_t *pay = ar.base + page + end - 8 - rec_payload_bytes(n);
        const uint32_t idx = (uint32_t)(i - r0);
        if (i < (int64_t)r0 || idx >= n) { bad = true; break; }
        const uint32_t code = (pay[idx >> 1] >> ((idx & 1) * 4)) & 15u;
        uint32_t op;
        if (state == 0) {
            const uint32_t src = code & 3u;
            if (src == 1) { state = 1; continue; }
            if (src == 2) { state = 2; continue; }
            op = 0; i--; j--;
        } else if (state == 1) {
            op = 1;
            if (code & 4u) state = 0;
            j--;
        } else {
            op = 2;
            if (code & 8u) state = 0;
            i--;
        }
        if (op == cur_op) {
            cur_len++;
        } else {
            if (cur_len) {
                if (cnt >= cap) { bad = true; break; }
                out[cnt++] = (cur_len << 2) | cur_op;
            }
            cur_op = op;
            cur_len = 1;
        }
    }
    if (!bad && cur_len) {
        if (cnt >= cap) bad = true;
        else out[cnt++] = (cur_len << 2) | cur_op;
    }
    nruns[x] = bad ? 0xffffffffu : cnt;
}

void launch_traceback(const HalfResult *res, const int32_t *half_ids, int64_t n, Arena arena,
                      const uint64_t *run_off, uint32_t *runs, uint32_t *nruns, hipStream_t st) {
    if (n <= 0) return;
    k_traceback<<<(unsigned)((n + 63) / 64), 64, 0, st>>>(res, half_ids, n, arena, run_off, runs, nruns);
}

// Final ops of an item: backward half (emission order already runs left to
// right), the anchor column, then the forward half reversed; adjacent equal
// runs merged.  Traced halves x2 (forward) and x2+1 (backward) of the item list.
__global__ void k_ops_assemble(const int32_t *__restrict__ item_ids, int64_t n, const uint64_t *__restrict__ run_off,
                               const uint32_t *__restrict__ runs, const uint32_t *__restrict__ nruns,
                               const uint64_t *__restrict__ ops_off, uint32_t *__restrict__ ops,
                               uint32_t *__restrict__ nops) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    (void)item_ids;
    const uint32_t *fr = runs + run_off[2 * x];
    const uint32_t *br = runs + run_off[2 * x + 1];
    const uint32_t nf = nruns[2 * x], nb = nruns[2 * x + 1];
    uint32_t *o = ops + ops_off[x];
    uint32_t c = 0;
    auto push = [&](uint32_t w) {
        if (c > 0 && (o[c - 1] & 3u) == (w & 3u)) o[c - 1] += w & ~3u;
        else o[c++] = w;
    };
    for (uint32_t y = 0; y < nb; y++) push(br[y]);
    push((1u << 2) | 0u);
    for (uint32_t y = nf; y > 0; y--) push(fr[y - 1]);
    nops[x] = c;
}

void launch_ops_assemble(const int32_t *item_ids, int64_t n, const uint64_t *run_off, const uint32_t *runs,
                         const uint32_t *nruns, const uint64_t *ops_off, uint32_t *ops, uint32_t *nops,
                         hipStream_t st) {
    if (n <= 0) return;
    k_ops_assemble<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(item_ids, n, run_off, runs, nruns, ops_off, ops, nops);
}

}  // namespace sfe
