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

#include "ydrop_common.h"

namespace sfe {

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = imax(v, __shfl_xor(v, m, 64));
    return v;
}

// Half tasks of the batch items: task 2x is the forward half, 2x+1 the backward half.
__global__ void k_make_tasks(const ExtItem *__restrict__ items, int64_t n, const int64_t *__restrict__ n_dev,
                             const UnitDesc *__restrict__ units, int64_t nt, HalfTask *__restrict__ tasks) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n_dev) n = *n_dev;
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
                       hipStream_t st, const int64_t *n_dev) {
    if (n <= 0) return;
    k_make_tasks<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(items, n, n_dev, units, nt, tasks);
}

// Clears the launch bookkeeping of a batch inside a recorded graph (a kernel,
// not a memset node): the chunk pool's bitmap and free count, the work-queue
// head and the run-arena head.
__global__ void k_sched_reset(uint32_t *__restrict__ bits, int32_t nwords, int32_t *__restrict__ avail,
                              int32_t avail0, unsigned int *__restrict__ qhead,
                              unsigned long long *__restrict__ run_head) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < nwords) bits[x] = 0u;
    if (x == 0) {
        *avail = avail0;
        *qhead = 0u;
        *run_head = 0ull;
    }
}

void launch_sched_reset(uint32_t *bits, int32_t nwords, int32_t *avail, int32_t avail0, unsigned int *qhead,
                        unsigned long long *run_head, hipStream_t st) {
    k_sched_reset<<<(unsigned)((nwords + 255) / 256), 256, 0, st>>>(bits, nwords, avail, avail0, qhead, run_head);
}

// ---------------------------------------------------------------------------
// Arena: page allocation and record writing (uniform across the wave or done
// by one thread of a workgroup)
// ---------------------------------------------------------------------------
struct PageCursor {
    uint64_t page;      // device address of the current allocation, ~0 if none
    uint32_t fill;      // bytes used by the header and records
    uint32_t size;      // bytes in the allocation
    uint32_t nrec;      // records in it (their index entries fill it from the end)
};

// Makes room for a record of `need` bytes for antidiagonal k (plus its index
// entry); returns false when the arena is exhausted.  Called by one thread.
__device__ __forceinline__ bool arena_reserve_1t(Arena &ar, PageCursor &pc, uint32_t need, int64_t k) {
    if (pc.page != ~0ull && pc.fill + need + 4 * (pc.nrec + 1) <= pc.size) return true;
    uint32_t pages = (need + ARENA_HDR + 4 + ARENA_PAGE - 1) / ARENA_PAGE;
    unsigned long long off = atomicAdd(ar.head, (unsigned long long)pages * ARENA_PAGE);
    if (off + (unsigned long long)pages * ARENA_PAGE > ar.bytes) return false;
    uint32_t *hdr = (uint32_t *)(ar.base + off);
    uint64_t prev = pc.page;
    hdr[0] = (uint32_t)prev;
    hdr[1] = (uint32_t)(prev >> 32);
    hdr[2] = (uint32_t)k;
    hdr[3] = pages;
    pc.page = (uint64_t)(ar.base + off);
    pc.fill = ARENA_HDR;
    pc.size = pages * ARENA_PAGE;
    pc.nrec = 0;
    return true;
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
        s_pc.page = ~0ull; s_pc.fill = 0; s_pc.size = 0; s_pc.nrec = 0;
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
        const uint32_t ng = nonempty ? (uint32_t)((hi - lo + 8) / 8) : 0u;
        if (t == 0) s_ok = arena_reserve_1t(ar, s_pc, 8 + 4 * ng, k) ? 1 : 0;
        __syncthreads();
        if (!s_ok) { status = HALF_ARENA_OVERFLOW; break; }
        uint32_t *rec = (uint32_t *)((uint8_t *)s_pc.page + s_pc.fill);
        const int thr = best - Y;
        const int c1 = (int)((k - 1) % 3), c2 = (int)((k + 1) % 3), c0 = (int)(k % 3);  // k-1, k-2, k
        const int e1 = (int)((k - 1) & 1), e0 = (int)(k & 1);
        if (nonempty) {
            for (int64_t i0 = lo + 8 * (int64_t)t; i0 <= hi; i0 += 8 * RING_T) {
                uint32_t word = 0;
                for (int u = 0; u < 8; u++) {
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
                    word |= code << (4 * u);
                    if (live) {
                        unsigned long long key = ((unsigned long long)(uint32_t)(H + 0x80000000u) << 32) |
                                                 (unsigned long long)(0xffffffffu - (uint32_t)i);
                        atomicMax(&s_best, key);
                        atomicMin(&s_min, (long long)i);
                        atomicMax(&s_max, (long long)i);
                    }
                }
                rec[2 + ((i0 - lo) >> 3)] = word;
            }
        }
        __syncthreads();
        uint32_t my_rec = s_pc.fill;
        if (t == 0) {
            rec[0] = nonempty ? (uint32_t)lo : 0u;
            rec[1] = rec_head_word(ng, 8);
            ((uint32_t *)((uint8_t *)s_pc.page + s_pc.size))[-(int)(s_pc.nrec + 1)] = s_pc.fill;
            s_pc.fill += 8 + 4 * ng;
            s_pc.nrec++;
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
                tb_end = my_rec;
            }
        }
        if (best >= SFE_SCORE_LIMIT) {
            status = HALF_SCORE_RANGE;
            __syncthreads();
            break;
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
// One wave per traced half.  The allocation holding the current record is
// staged in LDS (single-page allocations) so that each step costs two dependent
// LDS reads: the record's head through the page index, then the code word.
__global__ void __launch_bounds__(64) k_traceback(const HalfResult *__restrict__ res, const int32_t *__restrict__ half_ids,
                                                  int64_t nh, Arena ar, const uint64_t *__restrict__ run_off,
                                                  uint32_t *__restrict__ runs, uint32_t *__restrict__ nruns) {
    __shared__ uint32_t pbuf[ARENA_PAGE / 4];
    const int lane = threadIdx.x;
    const int64_t x = blockIdx.x;
    if (x >= nh) return;
    const int32_t h = half_ids[x];
    const HalfResult R = res[h];
    uint32_t *out = runs + run_off[x];
    int64_t i = R.i_end, j = R.j_end;
    if (i == 0 && j == 0) {
        if (lane == 0) nruns[x] = 0;
        return;
    }
    uint64_t page = R.tb_page;
    uint64_t prev = 0;
    int64_t k0 = 0;
    uint32_t size = 0;
    bool local = false;
    auto load = [&](uint64_t pgaddr) {
        const uint32_t *g = (const uint32_t *)pgaddr;
        prev = (uint64_t)g[0] | ((uint64_t)g[1] << 32);
        k0 = g[2];
        const uint32_t pages = g[3];
        size = pages * ARENA_PAGE;
        local = pages == 1;
        __syncthreads();
        if (local) {
            const uint4 *src = (const uint4 *)pgaddr;
            uint4 *dst = (uint4 *)pbuf;
            for (int q = lane; q < (int)(ARENA_PAGE / 16); q += 64) dst[q] = src[q];
        }
        __syncthreads();
    };
    auto rd = [&](uint32_t off) -> uint32_t {
        const uint32_t v = local ? pbuf[off >> 2] : ((const uint32_t *)page)[off >> 2];
        return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
    };
    load(page);
    const uint32_t cap = (uint32_t)(R.i_end + R.j_end + 1);
    int64_t guard = 2 * (i + j) + 4;
    bool bad = false;
    int state = 0;
    uint32_t cnt = 0, cur_op = 0xffffffffu, cur_len = 0;
    while (!(i == 0 && j == 0 && state == 0)) {
        if (--guard < 0 || i < 0 || j < 0) { bad = true; break; }
        const int64_t k = i + j;
        while (k < k0) {
            if (prev == ~0ull) { bad = true; break; }
            page = prev;
            load(page);
        }
        if (bad) break;
        const uint32_t xk = (uint32_t)(k - k0);
        if (4 * (xk + 1) + ARENA_HDR > size) { bad = true; break; }
        const uint32_t rec = rd(size - 4 * (xk + 1));
        const uint32_t r0 = rd(rec), w = rd(rec + 4);
        const uint32_t ng = w & 0xffffffu, G = w >> 24;
        const uint32_t idx = (uint32_t)(i - r0);
        if (i < (int64_t)r0 || G == 0 || G > 8 || idx / G >= ng) { bad = true; break; }
        const uint32_t code = (rd(rec + 8 + 4 * (idx / G)) >> (4 * (idx % G))) & 15u;
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
                if (lane == 0) out[cnt] = (cur_len << 2) | cur_op;
                cnt++;
            }
            cur_op = op;
            cur_len = 1;
        }
    }
    if (!bad && cur_len) {
        if (cnt >= cap) bad = true;
        else {
            if (lane == 0) out[cnt] = (cur_len << 2) | cur_op;
            cnt++;
        }
    }
    if (lane == 0) nruns[x] = bad ? 0xffffffffu : cnt;
}

void launch_traceback(const HalfResult *res, const int32_t *half_ids, int64_t n, Arena arena,
                      const uint64_t *run_off, uint32_t *runs, uint32_t *nruns, hipStream_t st) {
    if (n <= 0) return;
    k_traceback<<<(unsigned)n, 64, 0, st>>>(res, half_ids, n, arena, run_off, runs, nruns);
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
