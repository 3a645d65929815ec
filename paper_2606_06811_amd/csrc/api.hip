// api.hip -- the C ABI (include/sfe.h): contexts, the position table, and the
// host side of the speculative batched pipeline (Alg. 3 of the paper: a
// serial scan picks a batch, the GPU extends it, a serial commit keeps the
// result equal to the strict serial Alg. 1).
#include <algorithm>
#include <cmath>
#include <chrono>
#include <functional>
#include <memory>
#include <sys/mman.h>
#include <mutex>
#include <thread>
#include <atomic>
#include <exception>
#include <tuple>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "sfe_kernels.h"

using namespace sfe;

namespace {

struct SfeError {
    sfe_status st;
    std::string msg;
};

#define HIPCHK(x)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess)                                                                       \
            throw SfeError{SFE_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};          \
    } while (0)

void fail(sfe_status st, const std::string &m) { throw SfeError{st, m}; }

struct DBuf {
    void *p = nullptr;
    size_t n = 0;
    ~DBuf() { if (p) (void)hipFree(p); }
    void reset(size_t bytes) {
        if (p) { HIPCHK(hipFree(p)); p = nullptr; n = 0; }
        ensure(bytes);
    }
    void *ensure(size_t bytes) {
        if (bytes <= n && p) return p;
        if (p) { HIPCHK(hipFree(p)); p = nullptr; n = 0; }
        size_t b = std::max<size_t>(bytes, 256);
        if (hipMalloc(&p, b) != hipSuccess) { p = nullptr; fail(SFE_ENOMEM, "device allocation failed"); }
        n = b;
        return p;
    }
    template <class T> T *as() const { return (T *)p; }
};

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SeqSet {
    DBuf bases, nbits, sbits, nsum;
    int64_t total = 0;   // bases including padding
    SeqSetView view() const {
        return SeqSetView{(const uint32_t *)bases.p, (const uint32_t *)nbits.p, (const uint32_t *)sbits.p,
                          (const uint32_t *)nsum.p};
    }
};

}  // namespace

struct sfe_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string last_error;
    DBuf staging, cub_temp, tmp_a, tmp_b, tmp_c, tmp_d, tmp_e, counters;
    DBuf units_d, chunks_d, qdesc_d;
    DBuf hsp_raw, hsp_pass, hsp_sorted;
    DBuf items_d, tasks_d, hres_d, ids_d, aln_d, runoff_d, runs_d, nruns_d, opsoff_d, ops_d, nops_d, ring_d;
    DBuf sched_d;                       // scheduling words (kSchedBytes: heads, free count, counts)
    DBuf feat_unit, feat_key, feat_key2, feat_ids, feat_ids2, feat_okey, feat_range, feat_hsp, feat_out, feat_pred;
    DBuf busy_d;                        // bitmap of the traceback chunk pool
    int cu_count = 0;
    sfe_tuning tuning{};                // schedule knobs (wave_group_cap 0: one wave per half)
    int32_t pool_avail = 0;             // host copy of the pool's initial free count
    // traceback arenas: arena 0 holds the fused kernel's chunk pool and the
    // workgroup kernel's pages; a workgroup-kernel half that finds its arena
    // full is re-run into the next one (allocated twice as large on demand)
    std::vector<std::unique_ptr<DBuf>> arenas;
    DBuf arena_heads;
    int64_t arena_bytes = 0;            // size of arena 0
    SeqSet qplus, qminus;
    std::vector<QueryDesc> qdesc;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // per-call kernel accounting (reset by sfe_align)
    double ydrop_ms = 0, sx_ms = 0;
    int64_t ydrop_launches = 0, ydrop_cells = 0, sx_launches = 0, narrow_launches = 0;
    int64_t graph_launches = 0, graph_records = 0;
    // first launch of a batch recorded as a graph (tuning.use_graphs): the
    // executable graph, the launch it was recorded for (buffers, sizes,
    // scores), and the item and half counts it reads from device memory
    hipGraphExec_t round_exec = nullptr;
    std::vector<uint8_t> round_key;
    bool graphs_failed = false;         // recording failed once: plain stream launches from then on
    int64_t graph_counts[2] = {0, 0};
};

struct sfe_index {
    sfe_ctx *ctx = nullptr;
    int device = 0;
    SeqSet target;
    int64_t nt = 0;
    SeedDesc sd{};
    uint32_t K = 0;
    DBuf offsets, pos;
    int64_t n_valid = 0;
    int32_t max_abs_sub_guard = 0;
};

struct sfe_model {
    sfe_ctx *ctx = nullptr;             // must outlive the model (its stream runs the kernels)
    int device = 0;
    DBuf master, m, v, p16;             // FP32 master weights, Adam moments, BF16 copy
    DBuf part, sse, loss, x, t, ids, y, grad;
    int64_t step = 0;                   // Adam steps taken
};

namespace {

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) { (void)hipGetLastError(); return false; }
    return a.type == hipMemoryTypeDevice;
}

// Copy n bytes to the caller's buffer (host or device).
void copy_out(sfe_ctx *c, void *dst, const void *src_dev, size_t n) {
    if (n == 0) return;
    HIPCHK(hipMemcpyAsync(dst, src_dev, n, hipMemcpyDefault, c->stream));
}
void copy_in(sfe_ctx *c, void *dst_dev, const void *src, size_t n) {
    if (n == 0) return;
    HIPCHK(hipMemcpyAsync(dst_dev, src, n, hipMemcpyDefault, c->stream));
}
void sync(sfe_ctx *c) { HIPCHK(hipStreamSynchronize(c->stream)); }

// Elapsed time between the context's two events (both already complete).
double event_ms(sfe_ctx *c) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    return (double)ms;
}

unsigned grid(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int64_t padded(int64_t len) { return ((len + 63) / 64) * 64 + 64; }

// Packs sequences into a set; seq i starts at starts[i].  rc = 1 packs the
// reverse complements.
void pack_set(sfe_ctx *c, const sfe_seq *seqs, int32_t n, int rc, SeqSet &set, std::vector<int64_t> &starts) {
    starts.resize(n);
    int64_t total = 0;
    for (int32_t i = 0; i < n; i++) {
        if (seqs[i].length < 0 || (seqs[i].length > 0 && !seqs[i].residues)) fail(SFE_EINVAL, "bad sequence");
        if (seqs[i].length > (int64_t)0xffffffffLL - 64) fail(SFE_ERANGE, "sequence longer than 2^32 - 64");
        starts[i] = total;
        total += padded(seqs[i].length);
    }
    total += 64;
    set.total = total;
    set.bases.ensure((size_t)(total / 16 + 4) * 4);
    set.nbits.ensure((size_t)(total / 32 + 4) * 4);
    set.sbits.ensure((size_t)(total / 32 + 4) * 4);
    HIPCHK(hipMemsetAsync(set.bases.p, 0, (size_t)(total / 16 + 4) * 4, c->stream));
    HIPCHK(hipMemsetAsync(set.nbits.p, 0, (size_t)(total / 32 + 4) * 4, c->stream));
    HIPCHK(hipMemsetAsync(set.sbits.p, 0, (size_t)(total / 32 + 4) * 4, c->stream));
    int *bad = c->counters.ensure(64) ? (int *)c->counters.p : nullptr;
    HIPCHK(hipMemsetAsync(bad, 0, 4, c->stream));
    for (int32_t i = 0; i < n; i++) {
        int64_t len = seqs[i].length;
        if (len == 0) continue;
        const uint8_t *src = (const uint8_t *)seqs[i].residues;
        if (!is_device_ptr(src)) {
            c->staging.ensure((size_t)len);
            HIPCHK(hipMemcpyAsync(c->staging.p, src, (size_t)len, hipMemcpyHostToDevice, c->stream));
            src = c->staging.as<uint8_t>();
        }
        k_pack<<<grid((len + 31) / 32, 256), 256, 0, c->stream>>>(src, len, starts[i], rc, set.bases.as<uint32_t>(),
                                                                   set.nbits.as<uint32_t>(), set.sbits.as<uint32_t>(), bad);
        HIPCHK(hipGetLastError());
        if (src == c->staging.p) sync(c);   // staging is reused by the next sequence
    }
    // one summary bit per N-plane word, so that readers skip the plane where it is empty
    const int64_t nwords = total / 32 + 4;
    const int64_t nsw = nwords / 32 + 4;
    set.nsum.ensure((size_t)nsw * 4);
    HIPCHK(hipMemsetAsync(set.nsum.p, 0, (size_t)nsw * 4, c->stream));
    k_nsum<<<grid(nwords, 256), 256, 0, c->stream>>>(set.nbits.as<uint32_t>(), nwords, set.nsum.as<uint32_t>());
    HIPCHK(hipGetLastError());
    int hbad = 0;
    HIPCHK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (hbad) fail(SFE_EINVAL, "sequence holds a byte outside ACGTN / IUPAC letters");
}

SeedDesc parse_seed(const sfe_seed_spec *s) {
    if (!s || !s->pattern) fail(SFE_EINVAL, "null seed spec");
    SeedDesc d{};
    int span = (int)strlen(s->pattern);
    if (span < 1 || span > 32) fail(SFE_EINVAL, "seed span must be 1..32");
    if (s->pattern[0] != '1' || s->pattern[span - 1] != '1') fail(SFE_EINVAL, "seed must start and end with '1'");
    int w = 0;
    for (int i = 0; i < span; i++) {
        char ch = s->pattern[i];
        if (ch == '1') {
            if (w >= 14) fail(SFE_EINVAL, "seed weight above 14");
            d.care[w++] = i;
        } else if (ch != '0') {
            fail(SFE_EINVAL, "seed pattern holds a character other than 0/1");
        }
    }
    if (s->step < 1) fail(SFE_EINVAL, "step must be >= 1");
    if (s->transitions != 0 && s->transitions != 1) fail(SFE_EINVAL, "transitions must be 0 or 1");
    d.span = span;
    d.weight = w;
    d.transitions = s->transitions;
    d.step = s->step;
    return d;
}

ScoreDesc check_scoring(const sfe_scoring *s) {
    if (!s) fail(SFE_EINVAL, "null scoring");
    ScoreDesc d;
    for (int a = 0; a < 5; a++)
        for (int b = 0; b < 5; b++) {
            if (s->sub[a][b] <= -(1 << 15) || s->sub[a][b] >= (1 << 15)) fail(SFE_EINVAL, "|sub| must be < 2^15");
            d.sub[a][b] = s->sub[a][b];
        }
    if (s->gap_open < 0 || s->gap_open >= (1 << 20)) fail(SFE_EINVAL, "gap_open out of range");
    if (s->gap_extend <= 0 || s->gap_extend >= (1 << 15)) fail(SFE_EINVAL, "gap_extend out of range");
    if (s->xdrop < 0 || s->xdrop >= (1 << 29)) fail(SFE_EINVAL, "xdrop out of range");
    if (s->ydrop < 0 || s->ydrop >= (1 << 29)) fail(SFE_EINVAL, "ydrop out of range");
    d.gap_open = s->gap_open;
    d.gap_extend = s->gap_extend;
    d.xdrop = s->xdrop;
    d.hsp_thresh = s->hsp_thresh;
    d.ydrop = s->ydrop;
    d.gapped_thresh = s->gapped_thresh;
    return d;
}

int max_abs_sub(const ScoreDesc &d) {
    int m = 1;
    for (int a = 0; a < 5; a++)
        for (int b = 0; b < 5; b++) m = std::max(m, std::abs(d.sub[a][b]));
    return m;
}

template <class T>
void exclusive_sum(sfe_ctx *c, const T *in, T *out, int64_t n) {
    uint64_t *work = (uint64_t *)c->cub_temp.ensure((size_t)scan_work_words(n) * 8);
    scan_exclusive<T, T>(in, out, n, work, c->stream);
}

template <class K>
void sort_pairs(sfe_ctx *c, const K *kin, K *kout, const uint32_t *vin, uint32_t *vout, int64_t n, int end_bit) {
    void *temp = c->cub_temp.ensure((size_t)radix_temp_bytes(n, (int)sizeof(K)));
    radix_sort_pairs<K>(kin, kout, vin, vout, n, end_bit, temp, c->stream);
}

// Uploads the queries (both strands) and describes the (query, strand) units
// and 64-window chunks.
struct QueryLayout {
    std::vector<UnitDesc> units;
    std::vector<Chunk> chunks;
    std::vector<int64_t> starts;
};

void upload_queries(sfe_ctx *c, const sfe_seq *q, int32_t nq, int strands, int span, QueryLayout &L) {
    if (nq < 0 || (nq > 0 && !q)) fail(SFE_EINVAL, "bad query list");
    std::vector<int64_t> s2;
    pack_set(c, q, nq, 0, c->qplus, L.starts);
    pack_set(c, q, nq, 1, c->qminus, s2);
    c->qdesc.resize(nq);
    for (int32_t i = 0; i < nq; i++) c->qdesc[i] = QueryDesc{L.starts[i], q[i].length};
    L.units.clear();
    L.chunks.clear();
    for (int32_t i = 0; i < nq; i++)
        for (int s = 0; s < 2; s++) {
            if (!((strands >> s) & 1)) continue;
            UnitDesc u{L.starts[i], q[i].length, i, s};
            int32_t ui = (int32_t)L.units.size();
            L.units.push_back(u);
            int64_t nwin = q[i].length >= span ? q[i].length - span + 1 : 0;
            for (int64_t w = 0; w < nwin; w += 64) L.chunks.push_back(Chunk{ui, (int32_t)w});
        }
    c->units_d.ensure(std::max<size_t>(1, L.units.size()) * sizeof(UnitDesc));
    c->chunks_d.ensure(std::max<size_t>(1, L.chunks.size()) * sizeof(Chunk));
    c->qdesc_d.ensure(std::max<size_t>(1, c->qdesc.size()) * sizeof(QueryDesc));
    copy_in(c, c->units_d.p, L.units.data(), L.units.size() * sizeof(UnitDesc));
    copy_in(c, c->chunks_d.p, L.chunks.data(), L.chunks.size() * sizeof(Chunk));
    copy_in(c, c->qdesc_d.p, c->qdesc.data(), c->qdesc.size() * sizeof(QueryDesc));
}

// Sorts n HSPs (device) into the walking order and removes exact duplicates.
// Returns the unique count; result in c->hsp_sorted.  h must not live in the
// tmp_a..tmp_d scratch buffers, which the sort uses.
int64_t hsp_set(sfe_ctx *c, const sfe_hsp *h, int64_t n) {
    c->hsp_sorted.ensure((size_t)std::max<int64_t>(n, 1) * sizeof(sfe_hsp));
    if (n == 0) return 0;
    uint32_t *perm = (uint32_t *)c->tmp_a.ensure((size_t)n * 4);
    uint32_t *perm2 = (uint32_t *)c->tmp_b.ensure((size_t)n * 4);
    uint32_t *key = (uint32_t *)c->tmp_c.ensure((size_t)n * 4);
    uint32_t *key2 = (uint32_t *)c->tmp_d.ensure((size_t)n * 4);
    k_iota<<<grid(n, 256), 256, 0, c->stream>>>(perm, n);
    // least significant field first; radix sort is stable
    for (int field = 0; field < 6; field++) {
        k_hsp_key<<<grid(n, 256), 256, 0, c->stream>>>(h, perm, n, field, key);
        sort_pairs<uint32_t>(c, key, key2, perm, perm2, n, field == 3 ? 1 : 32);
        std::swap(perm, perm2);
    }
    uint32_t *flag = key, *dst = key2;
    k_hsp_unique_flags<<<grid(n, 256), 256, 0, c->stream>>>(h, perm, n, flag);
    exclusive_sum<uint32_t>(c, flag, dst, n);
    k_hsp_compact<<<grid(n, 256), 256, 0, c->stream>>>(h, perm, flag, dst, n, c->hsp_sorted.as<sfe_hsp>());
    uint32_t lastf = 0, lastd = 0;
    HIPCHK(hipMemcpyAsync(&lastf, flag + n - 1, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&lastd, dst + n - 1, 4, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    return (int64_t)lastd + lastf;
}

__global__ void k_hsp_filter(const sfe_hsp *__restrict__ in, int64_t n, int32_t thresh, sfe_hsp *__restrict__ out,
                             unsigned long long *__restrict__ cnt) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    sfe_hsp h = in[x];
    if (h.score >= thresh) out[atomicAdd(cnt, 1ull)] = h;
}

// ---------------------------------------------------------------------------
// One batch of gapped extensions (no commit): items -> alignments + ops.
// ---------------------------------------------------------------------------
// Host vector whose new elements are left uninitialised (buffers that a copy
// fills right away).
template <class T>
struct NoInit : std::allocator<T> {
    template <class U> struct rebind { using other = NoInit<U>; };
    NoInit() = default;
    template <class U> NoInit(const NoInit<U> &) {}
    template <class U, class... A> void construct(U *p, A &&...a) {
        if constexpr (sizeof...(A) == 0) ::new ((void *)p) U;
        else ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
using OpsVec = std::vector<uint32_t, NoInit<uint32_t>>;

struct BatchResult {
    std::vector<sfe_aln> alns;        // per item; ops_offset indexes `ops`, ops_len set for passing items
    OpsVec ops;
    std::vector<HalfResult> halves;   // per half (2x forward, 2x+1 backward of item x)
    int64_t reruns = 0;
    int64_t predicted = 0, mispredicted = 0;
};

// Default traceback arena, allocated on first use: half the device memory then
// free, and at least 32 GiB when the device has that much to spare (never
// more than the free memory less 2 GiB).  The codes of every long half in
// flight live there at once: a batch of a few thousand halves of 10^6
// antidiagonals holds a few hundred GB of codes at its peak, and a dry pool
// makes waves wait for chunks.
const int64_t kMinArena = (int64_t)32 << 30;
const int64_t kArenaFloor = (int64_t)64 << 20;
const int64_t kArenaSpare = (int64_t)2 << 30;
int64_t default_arena(sfe_ctx *) {
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    const int64_t f = (int64_t)freeb;
    const int64_t want = std::min(std::max(kMinArena, f / 2), std::max(f - kArenaSpare, f / 2));
    return std::max(want >> 18 << 18, kArenaFloor);
}

// Arena 0 of `bytes` when it fits (kept if already that large).  A request
// the device cannot hold is retried at half the size, down to 64 MiB and to
// no less than just above the current size (growth); below that the call
// fails with SFE_ENOMEM.
void ensure_arena(sfe_ctx *c, int64_t bytes) {
    if (c->arenas.empty()) c->arenas.emplace_back(new DBuf);
    DBuf &a = *c->arenas[0];
    if (c->arena_bytes >= bytes && a.p) return;
    const int64_t had = a.p ? c->arena_bytes : 0;
    if (a.p) {
        HIPCHK(hipFree(a.p));
        a.p = nullptr;
        a.n = 0;
        c->arena_bytes = 0;
    }
    for (int64_t b = std::max<int64_t>(bytes >> 18 << 18, (int64_t)1 << 18);;) {
        if (b <= had) fail(SFE_ENOMEM, "no device memory left for the traceback arena");
        if (hipMalloc(&a.p, (size_t)b) == hipSuccess) {
            a.n = (size_t)b;
            c->arena_bytes = b;
            break;
        }
        (void)hipGetLastError();
        a.p = nullptr;
        b = (b / 2) >> 18 << 18;
        if (b < kArenaFloor) fail(SFE_ENOMEM, "no device memory left for the traceback arena");
    }
    c->arena_heads.ensure(8 * 32);
}

// Grows arena 0 for a half whose codes did not fit with one wave in flight:
// four times larger, or as large as the free memory allows.
void grow_arena(sfe_ctx *c) {
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    const int64_t most = c->arena_bytes + (int64_t)freeb - kArenaSpare;
    ensure_arena(c, std::min<int64_t>(c->arena_bytes * 4, most));
}

void set_arena(sfe_ctx *c, int64_t bytes) {
    if (c->arena_bytes == bytes && !c->arenas.empty() && c->arenas[0]->p) return;
    c->arenas.clear();
    c->arenas.emplace_back(new DBuf);
    c->arenas[0]->reset((size_t)bytes);
    c->arena_bytes = bytes;
    c->arena_heads.ensure(8 * 32);
}

Arena arena_at(sfe_ctx *c, size_t ai) {
    if (ai >= 32) fail(SFE_ENOMEM, "traceback arenas exhausted");
    while (c->arenas.size() <= ai) c->arenas.emplace_back(new DBuf);
    const int64_t bytes = c->arena_bytes << ai;
    if (!c->arenas[ai]->p || (int64_t)c->arenas[ai]->n < bytes) c->arenas[ai]->ensure((size_t)bytes);
    return Arena{c->arenas[ai]->as<uint8_t>(), (uint64_t)bytes, c->arena_heads.as<unsigned long long>() + ai};
}

// Run arena of at least `runs` entries; the first `keep` entries survive a regrowth.
RunArena run_arena(sfe_ctx *c, uint64_t runs, uint64_t keep) {
    if (c->runs_d.n < runs * 4 || !c->runs_d.p) {
        DBuf grown;
        grown.ensure((size_t)std::max<uint64_t>(runs, 2 * (c->runs_d.n / 4)) * 4);
        if (keep) HIPCHK(hipMemcpyAsync(grown.p, c->runs_d.p, (size_t)keep * 4, hipMemcpyDeviceToDevice, c->stream));
        sync(c);
        std::swap(c->runs_d.p, grown.p);
        std::swap(c->runs_d.n, grown.n);
    }
    return RunArena{c->runs_d.as<uint32_t>(), (uint64_t)(c->runs_d.n / 4), c->sched_d.as<unsigned long long>()};
}

uint64_t run_head(sfe_ctx *c) {
    uint64_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, c->sched_d.p, 8, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    return h;
}
void set_run_head(sfe_ctx *c, uint64_t h) {
    HIPCHK(hipMemcpyAsync(c->sched_d.p, &h, 8, hipMemcpyHostToDevice, c->stream));
    sync(c);
}

// Blocks (one wave each) of the persistent fused kernel a compute unit takes at
// once, at most `wpc`: when occupancy alone allows more, each block also asks
// for the least amount of (unused) dynamic LDS that brings it down to wpc, so
// the grid spreads evenly -- wpc per CU, wpc / 4 per SIMD -- instead of piling
// onto the first CUs.  Returns that amount in `dyn`.
int persistent_per_cu(sfe_ctx *c, int C, bool perm, bool narrow, int wpc, size_t &dyn) {
    if (c->cu_count <= 0) {
        int n = 0;
        HIPCHK(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, c->device));
        c->cu_count = n;
    }
    auto blocks = [&](size_t d) { return ydrop_fused_blocks_per_cu(C, perm, narrow, true, d); };
    dyn = 0;
    int per_cu = blocks(0);
    if (per_cu <= 0) fail(SFE_EDEVICE, "occupancy query of the extension kernel failed");
    if (per_cu <= wpc) return per_cu;
    size_t lo = 0, hi = 65536;                  // blocks(lo) > wpc
    const int at_hi = blocks(hi);
    if (at_hi <= 0 || at_hi > wpc) {            // cannot get that low: take what the largest request gives
        if (at_hi > 0) { dyn = hi; per_cu = at_hi; }
        return per_cu;
    }
    while (hi - lo > 256) {
        const size_t mid = (lo + hi) / 2 / 256 * 256;
        const int b = blocks(mid);
        if (b > wpc || b <= 0) lo = mid;
        else hi = mid;
    }
    dyn = hi;
    return blocks(hi);
}

// Chunk pool over arena 0: chunks of 256 KB (smaller for a small arena, so
// that it holds at least 256 of them).  pool_layout only places it; make_pool
// also marks every chunk free.
ChunkPool pool_layout(sfe_ctx *c) {
    int shift = 18;
    while (shift > 12 && ((uint64_t)c->arena_bytes >> shift) < 256) shift--;
    const uint64_t nchunks = std::min<uint64_t>((uint64_t)c->arena_bytes >> shift, (uint64_t)1 << 30);
    const int32_t nwords = (int32_t)(nchunks / 32);
    if (nwords < 1) fail(SFE_EINVAL, "traceback arena too small");
    uint32_t *bits = (uint32_t *)c->busy_d.ensure((size_t)nwords * 4);
    int32_t *avail = (int32_t *)(c->sched_d.as<uint8_t>() + 16);
    c->pool_avail = nwords * 32;
    return ChunkPool{c->arenas[0]->as<uint8_t>(), bits, avail, nwords, shift};
}

ChunkPool make_pool(sfe_ctx *c) {
    ChunkPool pool = pool_layout(c);
    HIPCHK(hipMemsetAsync(pool.bits, 0, (size_t)pool.nwords * 4, c->stream));
    HIPCHK(hipMemcpyAsync(pool.avail, &c->pool_avail, 4, hipMemcpyHostToDevice, c->stream));
    return pool;
}

// Device words of the scheduling block c->sched_d: run-arena head (u64 at 0),
// work-queue head (u32 at 8), pool free count (i32 at 16), and the item and
// half counts a recorded launch reads (i64 at 24 and 32).
constexpr int kSchedBytes = 64;

template <class T> void key_put(std::vector<uint8_t> &k, const T &v) {
    const uint8_t *b = (const uint8_t *)&v;
    k.insert(k.end(), b, b + sizeof(T));
}

// First launch of a batch as one graph: clear the pool bitmap, the pool's free
// count, the work-queue head and the run-arena head (a kernel, no memset
// node), build the half tasks of the first n_dev[0] items, and run the fused
// extension over the first n_dev[1] halves of the queue.  The graph is
// recorded for item capacity icap and half capacity hcap and replayed, with the
// counts written to device memory first, for every later batch whose buffers,
// scores and launch shape are the same.  Returns false when recording or
// instantiation fails (the caller then launches on the stream).
bool launch_first_recorded(sfe_ctx *c, const sfe_index *idx, const ExtItem *items_d, int64_t n, int64_t icap,
                           HalfTask *tasks, const int32_t *ids, int64_t cnt, int64_t hcap, int C, bool perm,
                           bool narrow, bool persistent, int64_t count, SeqSetView T, SeqSetView Qp, SeqSetView Qm,
                           const ScoreDesc &sc, ChunkPool pool, RunArena ra, HalfResult *hres, int long_cap,
                           size_t dyn) {
    uint8_t *sched = c->sched_d.as<uint8_t>();
    unsigned int *qhead = (unsigned int *)(sched + 8);
    const int64_t *n_items = (const int64_t *)(sched + 24), *n_halves = (const int64_t *)(sched + 32);
    const int64_t grid = persistent ? count : hcap;
    std::vector<uint8_t> key;
    key_put(key, items_d); key_put(key, icap); key_put(key, tasks); key_put(key, ids); key_put(key, hcap);
    key_put(key, C); key_put(key, perm); key_put(key, narrow); key_put(key, persistent); key_put(key, grid);
    key_put(key, T); key_put(key, Qp); key_put(key, Qm); key_put(key, sc); key_put(key, pool); key_put(key, ra);
    key_put(key, hres); key_put(key, long_cap); key_put(key, dyn); key_put(key, idx->nt);
    key_put(key, c->units_d.p); key_put(key, sched);
    if (!c->round_exec || key != c->round_key) {
        if (c->round_exec) { (void)hipGraphExecDestroy(c->round_exec); c->round_exec = nullptr; }
        c->round_key.clear();
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        launch_sched_reset(pool.bits, pool.nwords, pool.avail, pool.nwords * 32, qhead, ra.head, c->stream);
        launch_make_tasks(items_d, icap, c->units_d.as<UnitDesc>(), idx->nt, tasks, c->stream, n_items);
        launch_ydrop_fused(C, perm, narrow, persistent, tasks, WorkQueue{ids, hcap, qhead, n_halves}, grid, T, Qp, Qm,
                           sc, pool, ra, hres, long_cap, dyn, c->stream);
        const hipError_t e0 = hipGetLastError();
        const hipError_t e1 = hipStreamEndCapture(c->stream, &g);
        hipGraphExec_t ge = nullptr;
        const hipError_t e2 = (e0 == hipSuccess && e1 == hipSuccess && g)
                                  ? hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) : hipErrorUnknown;
        if (g) (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            if (ge) (void)hipGraphExecDestroy(ge);
            (void)hipGetLastError();
            return false;
        }
        c->round_exec = ge;
        c->round_key = key;
        c->graph_records++;
    }
    c->graph_counts[0] = n;
    c->graph_counts[1] = cnt;
    HIPCHK(hipMemcpyAsync(sched + 24, c->graph_counts, 16, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    HIPCHK(hipGraphLaunch(c->round_exec, c->stream));
    c->graph_launches++;
    return true;
}

int64_t pow2_at_least(int64_t x, int64_t lo) {
    int64_t p = lo;
    while (p < x) p <<= 1;
    return p;
}

// Stages of a half: one wave with the caller's rows per lane, one wave with 8,
// a group of 4 waves with 2 and with 4 rows per lane, then the workgroup
// kernel with a ring of 4096 * 4^(stage - ST_RING) rows.
enum { ST_WAVE = 0, ST_WAVE8 = 1, ST_COOP2 = 2, ST_COOP4 = 3, ST_RING = 4 };

// Extends the 2n halves of the batch items and traces back every half that
// ends away from its anchor.  Fused kernel first (rows-per-lane window of
// cells_per_lane, then 8): a half whose band outgrows the window moves on,
// finally to the workgroup kernel (ring of 4096 * 4^(stage-2) rows) with the
// separate traceback.  A half that finds the chunk pool dry is re-run with
// four times fewer waves in flight (persistent schedule); with one wave, the
// arena grows.
//
// cost (optional): predicted log2(1 + cells) of every half.  The halves then
// start longest-predicted first (for the persistent schedule, the order of its
// queue); the output does not depend on it.
void run_batch(sfe_ctx *c, const sfe_index *idx, const std::vector<ExtItem> &items, const ScoreDesc &sc,
               int cells_per_lane, int schedule, BatchResult &out, const std::vector<float> *cost = nullptr,
               const std::vector<float> *extent = nullptr) {
    const int64_t n = (int64_t)items.size();
    out.alns.assign(n, sfe_aln{});
    out.ops.clear();
    if (n == 0) return;
    // recorded first launch: buffers sized for a power-of-two capacity, so that
    // later batches of up to that many items replay the same graph
    bool pending = c->tuning.use_graphs == 1 && !c->graphs_failed;
    const int64_t icap = pending ? pow2_at_least(n, 4096) : n;
    ExtItem *items_d = (ExtItem *)c->items_d.ensure((size_t)icap * sizeof(ExtItem));
    HalfTask *tasks = (HalfTask *)c->tasks_d.ensure((size_t)2 * icap * sizeof(HalfTask));
    HalfResult *hres = (HalfResult *)c->hres_d.ensure((size_t)2 * icap * sizeof(HalfResult));
    copy_in(c, items_d, items.data(), (size_t)n * sizeof(ExtItem));
    if (!pending) launch_make_tasks(items_d, n, c->units_d.as<UnitDesc>(), idx->nt, tasks, c->stream);
    SeqSetView T = idx->target.view(), Qp = c->qplus.view(), Qm = c->qminus.view();
    bool perm = true;                   // every score fits in int8: scores come from packed row profiles
    int smax = 0;
    for (int a = 0; a < 5; a++)
        for (int b = 0; b < 5; b++) {
            perm = perm && sc.sub[a][b] >= -128 && sc.sub[a][b] <= 127;
            smax = std::max(smax, std::abs(sc.sub[a][b]));
        }
    // packed 16-bit DP: live values relative to the Y-drop threshold stay below 2^15
    const bool narrow = perm && c->tuning.wide_scores == 0 &&
                        (int64_t)sc.ydrop + sc.gap_open + sc.gap_extend + 2 * (int64_t)smax + 512 <= 32767;
    const int64_t nh = 2 * n;
    std::vector<HalfResult> hr(nh);
    std::vector<uint64_t> roff(nh, 0);
    std::vector<uint32_t> nrun(nh, 0);
    std::vector<int> stage(nh, cells_per_lane < 8 ? ST_WAVE : ST_WAVE8), level(nh, 0);
    // a half still running after long_cap antidiagonals on one wave restarts on a
    // wave group; predicted longer: straight there
    const int long_cap = c->tuning.wave_group_cap;
    if (extent && long_cap > 0)
        for (int64_t h = 0; h < nh; h++)
            if ((*extent)[h] > std::log2((double)long_cap)) stage[h] = ST_COOP2;
    c->sched_d.ensure(kSchedBytes);
    if (c->arenas.empty() || !c->arenas[0]->p) ensure_arena(c, default_arena(c));
    if (!pending) set_run_head(c, 0);
    RunArena ra = run_arena(c, std::max<uint64_t>(1 << 12, (uint64_t)c->arena_bytes / 256), 0);
    // the work a recorded first launch does, on the stream instead
    auto eager_setup = [&] {
        launch_make_tasks(items_d, n, c->units_d.as<UnitDesc>(), idx->nt, tasks, c->stream);
        set_run_head(c, 0);
        pending = false;
    };
    std::vector<int32_t> todo;
    size_t ai = 0;                      // workgroup-kernel arena
    bool all = true, first = true;
    out.reruns = 0;
    out.predicted = out.mispredicted = 0;
    if (cost) {
        // two bins: halves predicted to compute at least 2^20 cells start first, longest first;
        // the rest keep batch order (neighbouring halves read neighbouring sequence, so the bulk
        // runs faster in that order than sorted by size)
        if ((int64_t)cost->size() != nh) fail(SFE_EINTERNAL, "cost vector size");
        const float kLong = 20.0f;
        todo.reserve(nh);
        for (int64_t h = 0; h < nh; h++)
            if ((*cost)[h] >= kLong) todo.push_back((int32_t)h);
        std::stable_sort(todo.begin(), todo.end(), [&](int32_t a, int32_t b) { return (*cost)[a] > (*cost)[b]; });
        for (int64_t h = 0; h < nh; h++)
            if (!((*cost)[h] >= kLong)) todo.push_back((int32_t)h);
        all = false;
    }
    for (;;) {
        std::vector<int32_t> group, rest;
        int sg = 1 << 20, lv = 1 << 20;
        if (all) {
            sg = stage[0];
            lv = 0;
        } else {
            for (int32_t h : todo) sg = std::min(sg, stage[h]);
            for (int32_t h : todo)
                if (stage[h] == sg) lv = std::min(lv, level[h]);
            for (int32_t h : todo) (stage[h] == sg && (sg >= ST_RING || level[h] == lv) ? group : rest).push_back(h);
        }
        if (pending && !(sg <= ST_WAVE8 && lv == 0)) eager_setup();
        const int32_t *ids = nullptr;
        int64_t cnt = nh;
        const int64_t hcap = pending ? pow2_at_least(all ? nh : (int64_t)group.size(), 8192) : 0;
        if (!all) {
            int32_t *idd = (int32_t *)c->ids_d.ensure(std::max<size_t>(group.size(), (size_t)hcap) * 4);
            copy_in(c, idd, group.data(), group.size() * 4);
            ids = idd;
            cnt = (int64_t)group.size();
            if (!first) out.reruns += cnt;
        }
        first = false;
        const bool fused = sg <= ST_COOP4;         // chunk pool + traceback in the same kernel
        bool recorded = false;                     // launched as a replay of the recorded graph
        int64_t nwaves = 0;
        uint64_t chunk_bytes = 0;
        Arena ar{};
        if (sg <= ST_WAVE8) {
            const int C = sg == ST_WAVE ? cells_per_lane : 8;
            const int64_t adaptive = c->tuning.adaptive_halves > 0 ? c->tuning.adaptive_halves : 131072;
            const bool persistent = schedule == SFE_SCHED_PERSISTENT || lv > 0 ||
                                    (schedule == SFE_SCHED_ADAPTIVE && cnt < adaptive);
            // persistent: a few waves per SIMD (long halves then share a SIMD with at most
            // one other wave); level L > 0 (the pool ran dry at level L - 1): 4^L times
            // fewer, pulling from the queue
            const int wpc = c->tuning.persist_waves_per_cu > 0 ? c->tuning.persist_waves_per_cu : 8;
            size_t dyn = 0;
            int64_t count = 0;
            if (persistent) {
                count = (int64_t)persistent_per_cu(c, C, perm, narrow, wpc, dyn) * c->cu_count;
                if (lv > 0) count = std::max<int64_t>(1, count >> std::min(62, 2 * lv));
            }
            nwaves = persistent ? count : 0;
            if (pending) {
                const ChunkPool pool = pool_layout(c);
                chunk_bytes = (uint64_t)1 << pool.shift;
                if (!launch_first_recorded(c, idx, items_d, n, icap, tasks, ids, cnt, hcap, C, perm, narrow,
                                           persistent, count, T, Qp, Qm, sc, pool, ra, hres, long_cap, dyn)) {
                    c->graphs_failed = true;
                    eager_setup();
                }
                pending = false;
                recorded = !c->graphs_failed;
            }
            if (!recorded) {
                ChunkPool pool = make_pool(c);
                chunk_bytes = (uint64_t)1 << pool.shift;
                unsigned int *qhead = (unsigned int *)(c->sched_d.as<uint8_t>() + 8);
                HIPCHK(hipMemsetAsync(qhead, 0, 4, c->stream));
                WorkQueue wq{ids, cnt, qhead, nullptr};
                HIPCHK(hipEventRecord(c->ev0, c->stream));
                launch_ydrop_fused(C, perm, narrow, persistent, tasks, wq, persistent ? count : cnt, T, Qp, Qm, sc,
                                   pool, ra, hres, long_cap, dyn, c->stream);
            }
        } else if (sg <= ST_COOP4) {
            // wave groups; level L > 0: at most 256 / 4^(L-1) halves in flight
            const int C = sg == ST_COOP2 ? 2 : 4;
            const int64_t slice = lv == 0 ? cnt : std::max<int64_t>(1, 256 >> std::min(62, 2 * (lv - 1)));
            nwaves = slice == 1 ? 1 : 0;
            HIPCHK(hipEventRecord(c->ev0, c->stream));
            for (int64_t o = 0; o < cnt; o += slice) {
                ChunkPool pool = make_pool(c);
                chunk_bytes = (uint64_t)1 << pool.shift;
                launch_ydrop_coop(C, perm, tasks, ids + o, std::min(slice, cnt - o), T, Qp, Qm, sc, pool, ra, hres,
                                  c->stream);
            }
        } else {
            // ring of 4096 * 4^s rows, s <= 6 (2^24 rows: the 16M-row band limit of the kernels)
            if (sg - ST_RING > 6) fail(SFE_EINTERNAL, "band width beyond 2^24 rows");
            const int64_t cap = (int64_t)4096 << (2 * (sg - ST_RING));
            ar = arena_at(c, ai);
            HIPCHK(hipMemsetAsync(ar.head, 0, 8, c->stream));
            // seven int32 rows of ring per half; as many halves per launch as half the free memory holds
            size_t freeb = 0, totalb = 0;
            HIPCHK(hipMemGetInfo(&freeb, &totalb));
            const int64_t per_half = 7 * cap * 4;
            const int64_t fit = std::max<int64_t>(1, (int64_t)(freeb / 2 + c->ring_d.n / 2) / per_half);
            const int64_t slice = std::min<int64_t>(cnt, fit);
            int32_t *ring = (int32_t *)c->ring_d.ensure((size_t)(slice * per_half));
            for (int64_t o = 0; o < cnt; o += slice)
                launch_ydrop_ring(tasks, ids + o, std::min(slice, cnt - o), T, Qp, Qm, sc, ar, ring, (int32_t)cap, hres,
                                  c->stream);
        }
        HIPCHK(hipGetLastError());
        if (fused) HIPCHK(hipEventRecord(c->ev1, c->stream));
        copy_out(c, hr.data(), hres, hr.size() * sizeof(HalfResult));
        sync(c);
        double launch_ms = 0;
        if (fused) {
            launch_ms = event_ms(c);
            c->ydrop_ms += launch_ms;
            c->ydrop_launches++;
            if (narrow && sg <= ST_WAVE8) c->narrow_launches++;
        }
        std::vector<int32_t> next = rest, traced;
        bool arena_full = false, runs_full = false, pool_full = false;
        auto check = [&](int32_t h) {
            const HalfResult &r = hr[h];
            if (fused) c->ydrop_cells += (int64_t)r.cells;
            switch (r.status) {
            case HALF_OK:
                if (fused) {
                    roff[h] = r.tb_page;
                    nrun[h] = r.tb_end;
                } else if (r.i_end || r.j_end) {
                    traced.push_back(h);
                }
                break;
            case HALF_WIDTH_OVERFLOW:
                // 384 -> 512 rows (one wave), 512 -> 1024 (wave group), then the workgroup kernel
                stage[h] = stage[h] == ST_WAVE ? ST_WAVE8 : stage[h] <= ST_COOP2 ? ST_COOP4 : stage[h] + 1;
                level[h] = 0;
                next.push_back(h);
                break;
            case HALF_LONG: stage[h] = std::max(stage[h], (int)ST_COOP2); level[h] = 0; next.push_back(h); break;
            case HALF_ARENA_OVERFLOW:
                if (fused) {
                    if (nwaves == 1) pool_full = true;    // one wave already: grow the arena
                    else level[h] = lv + 1;
                } else {
                    arena_full = true;
                }
                next.push_back(h);
                break;
            case HALF_RUNS_OVERFLOW: runs_full = true; next.push_back(h); break;
            case HALF_SCORE_RANGE: fail(SFE_ERANGE, "a gapped score reached 2^29");
            case HALF_TRACE_ERROR: fail(SFE_EINTERNAL, "traceback codes are inconsistent");
            default: fail(SFE_EINTERNAL, "unknown half status");
            }
        };
        if (all) for (int32_t h = 0; h < nh; h++) check(h);
        else for (int32_t h : group) check(h);
        if (runs_full) {
            // allocations past the end failed; everything handed out below cap is in use
            const uint64_t used = ra.cap;
            ra = run_arena(c, 2 * ra.cap, used);
            set_run_head(c, used);
        }
        if (!traced.empty()) {
            // workgroup-kernel halves: trace from the paged arena into the run arena
            uint64_t head = run_head(c);
            std::vector<uint64_t> off(traced.size());
            for (size_t x = 0; x < traced.size(); x++) {
                off[x] = head;
                head += (uint64_t)hr[traced[x]].i_end + (uint64_t)hr[traced[x]].j_end + 1;
            }
            ra = run_arena(c, head, run_head(c));
            set_run_head(c, head);
            int32_t *hid_d = (int32_t *)c->ids_d.ensure(traced.size() * 4);
            uint64_t *off_d = (uint64_t *)c->runoff_d.ensure(traced.size() * 8);
            uint32_t *cnt_d = (uint32_t *)c->nruns_d.ensure(traced.size() * 4);
            copy_in(c, hid_d, traced.data(), traced.size() * 4);
            copy_in(c, off_d, off.data(), traced.size() * 8);
            launch_traceback(hres, hid_d, (int64_t)traced.size(), ar, off_d, ra.base, cnt_d, c->stream);
            HIPCHK(hipGetLastError());
            std::vector<uint32_t> got(traced.size());
            copy_out(c, got.data(), cnt_d, got.size() * 4);
            sync(c);
            for (size_t x = 0; x < traced.size(); x++) {
                if (got[x] == 0xffffffffu) fail(SFE_EINTERNAL, "traceback records are inconsistent");
                roff[traced[x]] = off[x];
                nrun[traced[x]] = got[x];
            }
        }
        if (arena_full) ai++;
        if (pool_full) grow_arena(c);
        if (getenv("SFE_PROGRESS")) {
            int32_t kmax_seen = 0;      // antidiagonals of the longest half of the launch
            if (all) for (int32_t h = 0; h < nh; h++) kmax_seen = std::max(kmax_seen, hr[h].k_last);
            else for (int32_t h : group) kmax_seen = std::max(kmax_seen, hr[h].k_last);
            if (fused)
                fprintf(stderr, "[sfe]   launch: %s%s C=%d level %d, %lld halves, %lld waves, %llu KiB chunks, next %zu; "
                        "%.1f ms, longest half %d antidiagonals\n",
                        sg <= ST_WAVE8 ? "wave" : "wave group", recorded ? " (graph)" : "", sg == ST_WAVE ? cells_per_lane : sg == ST_WAVE8 ? 8
                        : sg == ST_COOP2 ? 2 : 4, lv, (long long)cnt, (long long)nwaves,
                        (unsigned long long)(chunk_bytes >> 10), next.size(), launch_ms, kmax_seen);
            else
                fprintf(stderr, "[sfe]   launch: workgroup stage %d, %lld halves, arena %zu%s, next %zu\n", sg,
                        (long long)cnt, ai, arena_full ? " (full)" : "", next.size());
        }
        all = false;
        todo.swap(next);
        if (todo.empty()) break;
    }
    if (cost) {
        for (int64_t h = 0; h < nh; h++) {
            out.predicted++;
            if (std::fabs((double)(*cost)[h] - std::log2(1.0 + (double)hr[h].cells)) > 2.0) out.mispredicted++;
        }
    }
    out.halves = hr;
    sfe_aln *aln_d = (sfe_aln *)c->aln_d.ensure((size_t)n * sizeof(sfe_aln));
    launch_assemble(items_d, n, c->units_d.as<UnitDesc>(), hres, T, Qp, Qm, sc, aln_d, c->stream);
    copy_out(c, out.alns.data(), aln_d, (size_t)n * sizeof(sfe_aln));
    sync(c);
    // edit operations of the passing items
    std::vector<int32_t> pass;
    std::vector<uint64_t> run_off;
    std::vector<uint32_t> nruns;
    for (int64_t x = 0; x < n; x++) {
        if (!(out.alns[x].flags & SFE_ALN_PASSED)) continue;
        pass.push_back((int32_t)x);
        for (int s = 0; s < 2; s++) {
            run_off.push_back(roff[2 * x + s]);
            nruns.push_back(nrun[2 * x + s]);
        }
    }
    if (pass.empty()) return;
    const int64_t np = (int64_t)pass.size();
    uint64_t *roff_d = (uint64_t *)c->runoff_d.ensure(run_off.size() * 8);
    uint32_t *nruns_d = (uint32_t *)c->nruns_d.ensure(nruns.size() * 4);
    copy_in(c, roff_d, run_off.data(), run_off.size() * 8);
    copy_in(c, nruns_d, nruns.data(), nruns.size() * 4);
    std::vector<uint64_t> ops_off(np);
    uint64_t ooff = 0;
    for (int64_t p = 0; p < np; p++) {
        ops_off[p] = ooff;
        ooff += (uint64_t)nruns[2 * p] + nruns[2 * p + 1] + 1;
    }
    uint64_t *ooff_d = (uint64_t *)c->opsoff_d.ensure((size_t)np * 8);
    uint32_t *ops_d = (uint32_t *)c->ops_d.ensure((size_t)ooff * 4);
    uint32_t *nops_d = (uint32_t *)c->nops_d.ensure((size_t)np * 4);
    copy_in(c, ooff_d, ops_off.data(), (size_t)np * 8);
    launch_ops_assemble(nullptr, np, roff_d, ra.base, nruns_d, ooff_d, ops_d, nops_d, c->stream);
    HIPCHK(hipGetLastError());
    // the edit runs stay at their reserved offsets (each item's slot may end in unused words)
    std::vector<uint32_t> nops(np);
    out.ops.resize(ooff);
    copy_out(c, nops.data(), nops_d, (size_t)np * 4);
    copy_out(c, out.ops.data(), ops_d, (size_t)ooff * 4);
    sync(c);
    for (int64_t p = 0; p < np; p++) {
        sfe_aln &a = out.alns[pass[p]];
        a.ops_offset = ops_off[p];
        a.ops_len = nops[p];
    }
}

// All seed hits of the uploaded units (L) into c->tmp_c, in (unit, q, t)
// order; returns their number.
int64_t seed_hits_device(sfe_ctx *c, const sfe_index *ix, const QueryLayout &L, sfe_hit **hits) {
    const int64_t nch = (int64_t)L.chunks.size();
    *hits = nullptr;
    if (nch == 0) return 0;
    uint64_t *cnt = (uint64_t *)c->tmp_d.ensure((size_t)nch * 64 * 8);
    uint64_t *off = (uint64_t *)c->tmp_e.ensure((size_t)nch * 64 * 8);
    SeqSetView Qp = c->qplus.view(), Qm = c->qminus.view();
    k_seed_count<<<(unsigned)nch, 64, 0, c->stream>>>(c->units_d.as<UnitDesc>(), c->chunks_d.as<Chunk>(), Qp, Qm,
                                                     ix->offsets.as<uint32_t>(), ix->sd, cnt);
    exclusive_sum<uint64_t>(c, cnt, off, nch * 64);
    uint64_t lastc = 0, lasto = 0;
    HIPCHK(hipMemcpyAsync(&lastc, cnt + nch * 64 - 1, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&lasto, off + nch * 64 - 1, 8, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    const int64_t total = (int64_t)(lastc + lasto);
    if (total == 0) return 0;
    sfe_hit *dst = (sfe_hit *)c->tmp_c.ensure((size_t)total * sizeof(sfe_hit));
    k_seed_emit<<<(unsigned)nch, 64, 0, c->stream>>>(c->units_d.as<UnitDesc>(), c->chunks_d.as<Chunk>(), Qp, Qm,
                                                    ix->offsets.as<uint32_t>(), ix->pos.as<uint32_t>(), ix->sd, off, dst);
    HIPCHK(hipGetLastError());
    *hits = dst;
    return total;
}

// Features (n x 16, device) of n device HSPs; the units of L give each
// (query, strand) its sequence; neighbours are HSPs of the same unit.
void compute_features(sfe_ctx *c, const sfe_index *ix, const QueryLayout &L, int32_t nq, const sfe_hsp *h, int64_t n,
                      float *F) {
    if (n <= 0) return;
    std::vector<int32_t> unit_of(2 * (size_t)std::max(nq, 1), -1);
    for (size_t u = 0; u < L.units.size(); u++) unit_of[2 * L.units[u].query_id + L.units[u].strand] = (int32_t)u;
    int32_t *uo = (int32_t *)c->feat_unit.ensure(unit_of.size() * 4);
    copy_in(c, uo, unit_of.data(), unit_of.size() * 4);
    uint64_t *key = (uint64_t *)c->feat_key.ensure((size_t)n * 8);
    uint64_t *key2 = (uint64_t *)c->feat_key2.ensure((size_t)n * 8);
    uint32_t *ids = (uint32_t *)c->feat_ids.ensure((size_t)n * 4);
    uint32_t *order = (uint32_t *)c->feat_ids2.ensure((size_t)n * 4);
    uint32_t *okey = (uint32_t *)c->feat_okey.ensure((size_t)n * 4);
    const size_t NU = std::max<size_t>(L.units.size(), 1);
    int64_t *range = (int64_t *)c->feat_range.ensure(2 * NU * 8);
    launch_hsp_anchor_keys(h, n, uo, key, ids, c->stream);
    sort_pairs<uint64_t>(c, key, key2, ids, order, n, 64);
    HIPCHK(hipMemsetAsync(range, 0, 2 * NU * 8, c->stream));
    launch_hsp_unit_ranges(h, uo, order, n, okey, range, range + NU, c->stream);
    launch_hsp_features(h, n, uo, c->units_d.as<UnitDesc>(), ix->target.view(), ix->nt, c->qplus.view(),
                        c->qminus.view(), order, okey, range, range + NU, F, c->stream);
    HIPCHK(hipGetLastError());
}

// Host copies of caller HSPs, checked against the sequences.
std::vector<sfe_hsp> checked_hsps(sfe_ctx *c, const sfe_index *ix, const sfe_seq *queries, int32_t nq,
                                  const sfe_hsp *hsps, int64_t n) {
    std::vector<sfe_hsp> hh((size_t)n);
    if (n == 0) return hh;
    if (!hsps) fail(SFE_EINVAL, "null hsps");
    HIPCHK(hipMemcpyAsync(hh.data(), hsps, (size_t)n * sizeof(sfe_hsp), hipMemcpyDefault, c->stream));
    sync(c);
    for (const sfe_hsp &h : hh) {
        if (h.query_id >= (uint32_t)nq || h.strand > 1 || h.len == 0) fail(SFE_EINVAL, "bad hsp");
        if ((int64_t)h.t0 + h.len > ix->nt || (int64_t)h.q0 + h.len > queries[h.query_id].length)
            fail(SFE_EINVAL, "hsp outside its sequences");
    }
    return hh;
}

// Bounding boxes of committed alignments of one unit, binned by target position.
struct BoxGrid {
    static const int SH = 14;
    std::vector<std::vector<int32_t>> bins;     // by target position >> SH
    std::vector<sfe_aln> boxes;
    void reset(int64_t nt) { bins.assign((size_t)(nt >> SH) + 2, {}); boxes.clear(); }
    void add(const sfe_aln &a) {
        int32_t id = (int32_t)boxes.size();
        boxes.push_back(a);
        for (int64_t b = a.t_start >> SH; b <= ((int64_t)a.t_end - 1) >> SH; b++) bins[(size_t)b].push_back(id);
    }
    bool inside(uint32_t t, uint32_t q) const {
        const size_t b = (size_t)(t >> SH);
        if (b >= bins.size() || bins[b].empty()) return false;
        for (int32_t id : bins[b]) {
            const sfe_aln &a = boxes[id];
            if (a.t_start <= t && t < a.t_end && a.q_start <= q && q < a.q_end) return true;
        }
        return false;
    }
};

// M runs of computed extensions, for "does (t, q) lie on an M column of one of
// them" tests: run start (target), length, and diagonal minus the alignment's
// start diagonal.  Each alignment keeps its runs in path order (so sorted by
// t and disjoint in t) and is entered in every 16 kbp target bin its box
// touches; a test reads the alignments of one bin, checks the box and
// binary-searches the run that could hold t.
struct RunStore {
    // one block of three arrays, 2 MiB aligned and advised as huge pages (the first
    // touch of hundreds of MB of 4 KiB pages costs more than the writes)
    struct Free { void operator()(uint8_t *p) const { free(p); } };
    std::unique_ptr<uint8_t[], Free> mem;
    uint32_t *rt = nullptr, *rl = nullptr;
    int32_t *rd = nullptr;
    size_t n = 0, cap = 0;
    // room for `more` further runs (new entries are left uninitialised; capacity doubles)
    void grow(size_t more) {
        if (n + more <= cap) return;
        const size_t nc = std::max(n + more, 2 * cap);
        const size_t huge = (size_t)2 << 20;
        const size_t bytes = (nc * 12 + huge - 1) / huge * huge;
        uint8_t *m = (uint8_t *)aligned_alloc(huge, bytes);
        if (!m) throw std::bad_alloc();
        (void)madvise(m, bytes, MADV_HUGEPAGE);
        uint32_t *t2 = (uint32_t *)m, *l2 = t2 + nc;
        int32_t *d2 = (int32_t *)(l2 + nc);
        if (n) {
            memcpy(t2, rt, n * 4);
            memcpy(l2, rl, n * 4);
            memcpy(d2, rd, n * 4);
        }
        mem.reset(m);
        rt = t2;
        rl = l2;
        rd = d2;
        cap = nc;
    }
};

// Paths (the M runs of one alignment each, in a RunStore) binned by target
// position; several sets may share one store.
struct PathSet {
    static const int SH = 14;
    struct Path { uint32_t t0, t1, q0, q1; size_t owner; size_t first; uint32_t count; };
    const RunStore *rs = nullptr;
    std::vector<Path> paths;
    std::vector<std::vector<uint32_t>> bins;    // by target position >> SH
    void reset(int64_t nt, const RunStore *store) {
        rs = store;
        paths.clear();
        bins.assign((size_t)(nt >> SH) + 2, {});
    }
    static uint32_t count_runs(const sfe_aln &a, const uint32_t *ops) {
        uint32_t n = 0;
        for (uint32_t x = 0; x < a.ops_len; x++) n += (ops[x] & 3u) == 0;
        return n;
    }
    // writes a's M runs at entry `first` of the store (sized for them)
    static void write_runs(RunStore &st, size_t first, const sfe_aln &a, const uint32_t *ops) {
        uint32_t t = a.t_start, q = a.q_start;
        const int64_t d0 = (int64_t)a.t_start - (int64_t)a.q_start;
        size_t r = first;
        for (uint32_t x = 0; x < a.ops_len; x++) {
            const uint32_t len = ops[x] >> 2, op = ops[x] & 3u;
            if (op == 0) {
                st.rt[r] = t;
                st.rl[r] = len;
                st.rd[r] = (int32_t)((int64_t)t - (int64_t)q - d0);
                r++;
                t += len;
                q += len;
            } else if (op == 1) {
                q += len;
            } else {
                t += len;
            }
        }
    }
    // a path over runs [first, first + count) of the store; returns its id, or -1 if empty
    int64_t link(const sfe_aln &a, size_t first, uint32_t count, size_t owner) {
        if (count == 0 || a.t_end <= a.t_start) return -1;
        const uint32_t id = (uint32_t)paths.size();
        paths.push_back(Path{a.t_start, a.t_end, a.q_start, a.q_end, owner, first, count});
        for (uint32_t b = a.t_start >> SH; b <= (a.t_end - 1) >> SH; b++) bins[b].push_back(id);
        return id;
    }
    // visits the owners of the paths that have (t, q) on an M column and pass `pre` (cheap,
    // tested before the search); stops when `found` returns true, and returns whether it did
    template <class Pre, class Found>
    bool search(uint32_t t, uint32_t q, Pre pre, Found found) const {
        const size_t b = (size_t)(t >> SH);
        if (b >= bins.size()) return false;
        const uint32_t *rt = rs->rt, *rl = rs->rl;
        const int32_t *rd = rs->rd;
        for (uint32_t id : bins[b]) {
            const Path &P = paths[id];
            if (t < P.t0 || t >= P.t1 || q < P.q0 || q >= P.q1 || !pre(P.owner)) continue;
            // last run starting at or before t
            size_t lo = P.first, hi = P.first + P.count;
            while (hi - lo > 1) {
                const size_t mid = (lo + hi) / 2;
                if (rt[mid] <= t) lo = mid;
                else hi = mid;
            }
            if (rt[lo] <= t && t < rt[lo] + rl[lo] &&
                (int64_t)t - (int64_t)q - ((int64_t)P.t0 - (int64_t)P.q0) == (int64_t)rd[lo] && found(P.owner))
                return true;
        }
        return false;
    }
    // (t, q) on an M column of a path whose owner passes `pre` and then `post`
    template <class Pre, class Post>
    bool contains(uint32_t t, uint32_t q, Pre pre, Post post) const { return search(t, q, pre, post); }
};

// Every passing extension's M runs of one (query, strand) unit, owner = its
// position in the walking order, in `set`; the committed ones also in `done`
// (same runs).  Alg. 1's containment test reads `done`; the deferral rule
// reads `set`, restricted to the extensions still waiting for commit.
struct UnitPaths {
    RunStore runs;
    PathSet set, done;
    std::vector<size_t> run_first;      // per position: its runs in the store
    std::vector<uint32_t> run_count;
    std::vector<uint8_t> committed;
    void reset(int64_t nt, size_t n) {
        runs.mem.reset();
        runs.rt = runs.rl = nullptr;
        runs.rd = nullptr;
        runs.n = runs.cap = 0;
        set.reset(nt, &runs);
        done.reset(nt, &runs);
        run_first.assign(n, 0);
        run_count.assign(n, 0);
        committed.assign(n, 0);
    }
    // extension p, whose runs were written at [first, first + count)
    void add(const sfe_aln &a, size_t first, uint32_t count, size_t p) {
        run_first[p] = first;
        run_count[p] = count;
        set.link(a, first, count, p);
    }
    void commit(const sfe_aln &a, size_t p) {
        committed[p] = 1;
        done.link(a, run_first[p], run_count[p], p);
    }
    bool in_committed(uint32_t t, uint32_t q) const {
        return done.contains(t, q, [](size_t) { return true; }, [](size_t) { return true; });
    }
};

// f(u, thread) for every unit u in [0, n) on up to 16 host threads; the
// units of the commit bookkeeping share nothing.  The first exception a
// thread raises is raised again here.
template <class F>
void for_each_unit(size_t n, F &&f) {
    const size_t hw = std::max<size_t>(1, std::thread::hardware_concurrency());
    const size_t T = std::min<size_t>(n, std::min<size_t>(hw, 16));
    if (T <= 1) {
        for (size_t u = 0; u < n; u++) f(u, (size_t)0);
        return;
    }
    std::atomic<size_t> next{0};
    std::exception_ptr err;
    std::mutex mu;
    std::vector<std::thread> th;
    for (size_t t = 0; t < T; t++)
        th.emplace_back([&, t] {
            try {
                for (size_t u = next++; u < n; u = next++) f(u, t);
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu);
                if (!err) err = std::current_exception();
                next = n;
            }
        });
    for (auto &x : th) x.join();
    if (err) std::rethrow_exception(err);
}

sfe_status guard(sfe_ctx *c, const std::function<void()> &f) {
    try {
        (void)hipGetLastError();        // an error left by an unrelated earlier call is not this call's
        if (c) HIPCHK(hipSetDevice(c->device));
        f();
        return SFE_OK;
    } catch (const SfeError &e) {
        if (c) c->last_error = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        if (c) c->last_error = "host allocation failed";
        return SFE_ENOMEM;
    } catch (...) {
        if (c) c->last_error = "internal error";
        return SFE_EINTERNAL;
    }
}

}  // namespace

// Model file: a 32-byte header (magic "SFEMLP\0\0", u32 version 1, u32 layout 1
// = 16-64-64-64-4 ReLU network with the parameter order of sfe.h, u32
// parameter count, u32 zero, i64 Adam steps taken), the FP32 master
// parameters, the two Adam moment vectors, then a u64 FNV-1a hash of every
// preceding byte.  Little-endian.
namespace {
const char kModelMagic[8] = {'S', 'F', 'E', 'M', 'L', 'P', 0, 0};
const size_t kModelHeader = 32;
const size_t kModelBytes = kModelHeader + 3 * (size_t)SFE_MLP_NPARAMS * 4 + 8;

uint64_t fnv1a(const uint8_t *p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; i++) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Reads and checks a model file; SFE_EIO when it cannot be read, SFE_EINVAL
// when it is not a model of this layout.
sfe_status read_model_file(const char *path, std::vector<uint8_t> &buf, std::string &why) {
    FILE *f = fopen(path, "rb");
    if (!f) { why = std::string("cannot open ") + path; return SFE_EIO; }
    buf.assign(kModelBytes + 1, 0);
    const size_t got = fread(buf.data(), 1, buf.size(), f);
    const bool err = ferror(f) != 0;
    fclose(f);
    if (err) { why = std::string("cannot read ") + path; return SFE_EIO; }
    if (got != kModelBytes) { why = "model file has the wrong size"; return SFE_EINVAL; }
    buf.resize(kModelBytes);
    uint32_t ver = 0, layout = 0, np = 0, zero = 0;
    memcpy(&ver, buf.data() + 8, 4);
    memcpy(&layout, buf.data() + 12, 4);
    memcpy(&np, buf.data() + 16, 4);
    memcpy(&zero, buf.data() + 20, 4);
    int64_t steps = 0;
    memcpy(&steps, buf.data() + 24, 8);
    if (memcmp(buf.data(), kModelMagic, 8) != 0) { why = "not a model file (magic)"; return SFE_EINVAL; }
    if (ver != 1 || layout != 1 || np != SFE_MLP_NPARAMS || zero != 0 || steps < 0) {
        why = "model file of another version, layout or size";
        return SFE_EINVAL;
    }
    uint64_t h = 0;
    memcpy(&h, buf.data() + kModelBytes - 8, 8);
    if (h != fnv1a(buf.data(), kModelBytes - 8)) { why = "model file checksum mismatch"; return SFE_EINVAL; }
    return SFE_OK;
}
}  // namespace

// Working memory of sfe_model_grad_noalloc, one fixed array per device: the
// sample ids, then per-block squared errors, then per-block partial gradients
// (64 samples per block) for up to SFE_NOALLOC_MAX_SAMPLES samples -- about
// 10 MB, held by every device the library runs on until the process ends.
// Host code never passes the array's name to a kernel: it takes the device
// address from hipGetSymbolAddress, once per device, when a context is made.
namespace {
constexpr size_t kNoAllocBlocks = (SFE_NOALLOC_MAX_SAMPLES + 63) / 64;
constexpr size_t kScratchIds = (size_t)SFE_NOALLOC_MAX_SAMPLES * 4;
constexpr size_t kScratchSse = (kNoAllocBlocks * 4 + 255) / 256 * 256;
constexpr size_t kScratchPart = kNoAllocBlocks * SFE_MLP_NPARAMS * 4;
constexpr size_t kScratchBytes = kScratchIds + kScratchSse + kScratchPart;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
void scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) fail(SFE_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return;
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch[device] = (uint8_t *)ptr;
}

uint8_t *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

sfe_status sfe_ctx_create(int device, void *hip_stream, sfe_ctx **out) {
    if (!out) return SFE_EINVAL;
    *out = nullptr;
    sfe_ctx *c = new (std::nothrow) sfe_ctx;
    if (!c) return SFE_ENOMEM;
    c->device = device;
    sfe_status st = guard(c, [&] {
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        HIPCHK(upload_encoding_table(c->stream));
        scratch_setup(device);
        HIPCHK(hipEventCreate(&c->ev0));
        HIPCHK(hipEventCreate(&c->ev1));
        c->counters.ensure(64);
        sync(c);
    });
    if (st != SFE_OK) {
        delete c;
        return st;
    }
    *out = c;
    return SFE_OK;
}

void sfe_ctx_destroy(sfe_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->round_exec) (void)hipGraphExecDestroy(c->round_exec);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

sfe_status sfe_build_index(sfe_ctx *c, const sfe_seq *target, const sfe_seed_spec *seed, sfe_index **out) {
    if (!c || !target || !out) return SFE_EINVAL;
    *out = nullptr;
    sfe_index *ix = new (std::nothrow) sfe_index;
    if (!ix) return SFE_ENOMEM;
    sfe_status st = guard(c, [&] {
        ix->ctx = c;
        ix->device = c->device;
        ix->sd = parse_seed(seed);
        std::vector<int64_t> starts;
        pack_set(c, target, 1, 0, ix->target, starts);
        ix->nt = target->length;
        const SeedDesc &sd = ix->sd;
        ix->K = 1u << (2 * sd.weight);
        int64_t nslots = ix->nt >= sd.span ? (ix->nt - sd.span) / sd.step + 1 : 0;
        uint32_t *keys = (uint32_t *)c->tmp_a.ensure((size_t)std::max<int64_t>(nslots, 1) * 4);
        uint32_t *pos0 = (uint32_t *)c->tmp_b.ensure((size_t)std::max<int64_t>(nslots, 1) * 4);
        uint32_t *keys2 = (uint32_t *)c->tmp_c.ensure((size_t)std::max<int64_t>(nslots, 1) * 4);
        ix->pos.ensure((size_t)std::max<int64_t>(nslots, 1) * 4);
        ix->offsets.ensure(((size_t)ix->K + 1) * 4);
        if (nslots > 0) {
            k_index_keys<<<grid(nslots, 256), 256, 0, c->stream>>>(ix->target.view(), nslots, sd.step, sd, ix->K, keys, pos0);
            sort_pairs<uint32_t>(c, keys, keys2, pos0, ix->pos.as<uint32_t>(), nslots, 2 * sd.weight + 1);
        }
        k_offsets<<<grid(nslots + 1, 256), 256, 0, c->stream>>>(keys2, nslots, ix->K, ix->offsets.as<uint32_t>());
        HIPCHK(hipGetLastError());
        uint32_t nv = 0;
        HIPCHK(hipMemcpyAsync(&nv, ix->offsets.as<uint32_t>() + ix->K, 4, hipMemcpyDeviceToHost, c->stream));
        sync(c);
        ix->n_valid = nv;
    });
    if (st != SFE_OK) {
        delete ix;
        return st;
    }
    *out = ix;
    return SFE_OK;
}

void sfe_index_destroy(sfe_index *ix) {
    if (!ix) return;
    (void)hipSetDevice(ix->device);
    delete ix;
    (void)hipGetLastError();
}

sfe_status sfe_seed_hits(sfe_ctx *c, const sfe_index *ix, const sfe_seq *queries, int32_t nq, int32_t strands,
                         sfe_hit *out, int64_t cap, int64_t *n_hits) {
    if (!c || !ix || !n_hits) return SFE_EINVAL;
    return guard(c, [&] {
        if (strands == 0) strands = 3;
        if (strands < 0 || strands > 3) fail(SFE_EINVAL, "strands must be 1, 2 or 3");
        QueryLayout L;
        upload_queries(c, queries, nq, strands, ix->sd.span, L);
        int64_t nch = (int64_t)L.chunks.size();
        *n_hits = 0;
        if (nch == 0) return;
        uint64_t *cnt = (uint64_t *)c->tmp_d.ensure((size_t)nch * 64 * 8);
        uint64_t *off = (uint64_t *)c->tmp_e.ensure((size_t)nch * 64 * 8);
        SeqSetView Qp = c->qplus.view(), Qm = c->qminus.view();
        k_seed_count<<<(unsigned)nch, 64, 0, c->stream>>>(c->units_d.as<UnitDesc>(), c->chunks_d.as<Chunk>(), Qp, Qm,
                                                         ix->offsets.as<uint32_t>(), ix->sd, cnt);
        exclusive_sum<uint64_t>(c, cnt, off, nch * 64);
        uint64_t lastc = 0, lasto = 0;
        HIPCHK(hipMemcpyAsync(&lastc, cnt + nch * 64 - 1, 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(&lasto, off + nch * 64 - 1, 8, hipMemcpyDeviceToHost, c->stream));
        sync(c);
        int64_t total = (int64_t)(lastc + lasto);
        *n_hits = total;
        if (total > cap) fail(SFE_ECAPACITY, "hit buffer too small");
        if (total == 0) return;
        if (!out) fail(SFE_EINVAL, "null output");
        sfe_hit *dst = out;
        bool dev = is_device_ptr(out);
        if (!dev) dst = (sfe_hit *)c->tmp_c.ensure((size_t)total * sizeof(sfe_hit));
        k_seed_emit<<<(unsigned)nch, 64, 0, c->stream>>>(c->units_d.as<UnitDesc>(), c->chunks_d.as<Chunk>(), Qp, Qm,
                                                        ix->offsets.as<uint32_t>(), ix->pos.as<uint32_t>(), ix->sd, off, dst);
        HIPCHK(hipGetLastError());
        if (!dev) copy_out(c, out, dst, (size_t)total * sizeof(sfe_hit));
        sync(c);
    });
}

sfe_status sfe_ungapped_xdrop(sfe_ctx *c, const sfe_index *ix, const sfe_seq *queries, int32_t nq, const sfe_hit *hits,
                              int64_t n, const sfe_scoring *scp, int32_t flags, sfe_hsp *out, int64_t cap,
                              int64_t *n_hsps) {
    if (!c || !ix || !n_hsps || n < 0) return SFE_EINVAL;
    return guard(c, [&] {
        ScoreDesc sc = check_scoring(scp);
        QueryLayout L;
        upload_queries(c, queries, nq, 3, ix->sd.span, L);
        *n_hsps = 0;
        if (n == 0) return;
        if (!hits) fail(SFE_EINVAL, "null hits");
        // validate the hits on the host copy
        std::vector<sfe_hit> hh((size_t)n);
        HIPCHK(hipMemcpyAsync(hh.data(), hits, (size_t)n * sizeof(sfe_hit), hipMemcpyDefault, c->stream));
        sync(c);
        for (const sfe_hit &h : hh) {
            if (h.query_id >= (uint32_t)nq || h.strand > 1) fail(SFE_EINVAL, "hit names an unknown query or strand");
            if ((int64_t)h.t + ix->sd.span > ix->nt || (int64_t)h.q + ix->sd.span > queries[h.query_id].length)
                fail(SFE_EINVAL, "hit window outside its sequence");
        }
        sfe_hit *hd = (sfe_hit *)c->tmp_e.ensure((size_t)n * sizeof(sfe_hit));
        copy_in(c, hd, hh.data(), (size_t)n * sizeof(sfe_hit));
        sfe_hsp *raw = (sfe_hsp *)c->hsp_raw.ensure((size_t)n * sizeof(sfe_hsp));
        int *err = (int *)c->counters.as<char>() + 8;
        HIPCHK(hipMemsetAsync(err, 0, 4, c->stream));
        launch_xdrop_raw(hd, n, c->qdesc_d.as<QueryDesc>(), nq, ix->target.view(), 0, ix->nt, c->qplus.view(),
                         c->qminus.view(), sc, ix->sd.span, raw, err, c->stream);
        HIPCHK(hipGetLastError());
        int herr = 0;
        HIPCHK(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, c->stream));
        sync(c);
        if (herr) fail(SFE_ERANGE, "an ungapped score reached 2^29");
        if (flags & SFE_XDROP_RAW) {
            *n_hsps = n;
            if (n > cap) fail(SFE_ECAPACITY, "hsp buffer too small");
            if (!out) fail(SFE_EINVAL, "null output");
            copy_out(c, out, raw, (size_t)n * sizeof(sfe_hsp));
            sync(c);
            return;
        }
        sfe_hsp *pass = (sfe_hsp *)c->hsp_pass.ensure((size_t)n * sizeof(sfe_hsp));
        unsigned long long *cnt = c->counters.as<unsigned long long>();
        HIPCHK(hipMemsetAsync(cnt, 0, 8, c->stream));
        k_hsp_filter<<<grid(n, 256), 256, 0, c->stream>>>(raw, n, sc.hsp_thresh, pass, cnt);
        unsigned long long np = 0;
        HIPCHK(hipMemcpyAsync(&np, cnt, 8, hipMemcpyDeviceToHost, c->stream));
        sync(c);
        int64_t nu = hsp_set(c, pass, (int64_t)np);
        *n_hsps = nu;
        if (nu > cap) fail(SFE_ECAPACITY, "hsp buffer too small");
        if (nu && !out) fail(SFE_EINVAL, "null output");
        copy_out(c, out, c->hsp_sorted.p, (size_t)nu * sizeof(sfe_hsp));
        sync(c);
    });
}

sfe_status sfe_gapped_ydrop(sfe_ctx *c, const sfe_index *ix, const sfe_seq *queries, int32_t nq, const sfe_hsp *hsps,
                            int64_t n, const sfe_scoring *scp, sfe_aln *out, uint32_t *ops, int64_t ops_cap,
                            int64_t *n_ops) {
    if (!c || !ix || !n_ops || n < 0) return SFE_EINVAL;
    return guard(c, [&] {
        ScoreDesc sc = check_scoring(scp);
        QueryLayout L;
        upload_queries(c, queries, nq, 3, ix->sd.span, L);
        *n_ops = 0;
        if (n == 0) return;
        if (!hsps || !out) fail(SFE_EINVAL, "null hsps or output");
        std::vector<sfe_hsp> hh = checked_hsps(c, ix, queries, nq, hsps, n);
        std::vector<ExtItem> items((size_t)n);
        for (int64_t x = 0; x < n; x++) {
            const sfe_hsp &h = hh[x];
            uint32_t off = (h.len - 1) / 2;
            items[x] = ExtItem{h.t0 + off, h.q0 + off, (int32_t)(2 * h.query_id + h.strand), 0};
        }
        BatchResult br;
        run_batch(c, ix, items, sc, 6, SFE_SCHED_PLAIN, br);
        // edit runs packed in item order
        std::vector<uint32_t> packed;
        for (sfe_aln &a : br.alns) {
            if (!(a.flags & SFE_ALN_PASSED)) continue;
            const uint64_t src = a.ops_offset;
            a.ops_offset = packed.size();
            packed.insert(packed.end(), br.ops.begin() + (ptrdiff_t)src, br.ops.begin() + (ptrdiff_t)(src + a.ops_len));
        }
        int64_t need = (int64_t)packed.size();
        *n_ops = need;
        if (need > ops_cap) fail(SFE_ECAPACITY, "ops buffer too small");
        if (need && !ops) fail(SFE_EINVAL, "null ops");
        copy_out(c, out, br.alns.data(), (size_t)n * sizeof(sfe_aln));
        copy_out(c, ops, packed.data(), (size_t)need * 4);
        sync(c);
    });
}

sfe_status sfe_align_opts_resolve(const sfe_align_opts *in, sfe_align_opts *out) {
    if (!out) return SFE_EINVAL;
    sfe_align_opts o{};
    if (in) o = *in;
    if (o.strands == 0) o.strands = 3;
    if (o.strands < 1 || o.strands > 3) return SFE_EINVAL;
    if (o.schedule < SFE_SCHED_PLAIN || o.schedule > SFE_SCHED_BINNED) return SFE_EINVAL;
    if (o.policy != SFE_POLICY_DEFER && o.policy != SFE_POLICY_PREFIX) return SFE_EINVAL;
    if (o.arena_bytes < 0) return SFE_EINVAL;
    if (o.filter != SFE_FILTER_XDROP && o.filter != SFE_FILTER_YDROP) return SFE_EINVAL;
    if (o.max_cells_per_lane == 0) o.max_cells_per_lane = 6;
    if (o.max_cells_per_lane < 0) return SFE_EINVAL;
    o.max_cells_per_lane = std::min(8, std::max(2, o.max_cells_per_lane));
    if (o.near_band == 0) o.near_band = 32;
    if (o.near_band < 0) o.near_band = -1;
    if (o.round_k < 0) return SFE_EINVAL;
    if (o.round_k == 0) {
        // Every HSP of a (query, strand) that nothing defers enters the batch: with the
        // nearness rule on, the rule keeps each region's later HSPs back; without it a
        // batch would hold every HSP of a region at once, so it is capped like Alg. 3's.
        const bool rule_on = o.policy == SFE_POLICY_DEFER && o.near_band > 0;
        o.round_k = rule_on ? (1 << 20) : 256;
    }
    *out = o;
    return SFE_OK;
}

sfe_status sfe_align(sfe_ctx *c, const sfe_index *ix, const sfe_seq *queries, int32_t nq, const sfe_scoring *scp,
                     const sfe_align_opts *opts, sfe_aln *out, int64_t cap, int64_t *n_alns, uint32_t *ops,
                     int64_t ops_cap, int64_t *n_ops, sfe_stats *stats) {
    if (!c || !ix || !n_alns || !n_ops) return SFE_EINVAL;
    return guard(c, [&] {
        const double t0 = now_ms();
        ScoreDesc sc = check_scoring(scp);
        sfe_align_opts o{};
        if (sfe_align_opts_resolve(opts, &o) != SFE_OK) fail(SFE_EINVAL, "invalid sfe_align options");
        const int strands = o.strands;
        const int64_t K = o.round_k;
        const int cpl = o.max_cells_per_lane;
        if (o.arena_bytes > 0) set_arena(c, std::max<int64_t>(o.arena_bytes, 2 * ARENA_PAGE));
        sfe_stats st{};
        c->ydrop_ms = c->sx_ms = 0;
        c->ydrop_launches = c->ydrop_cells = c->sx_launches = c->narrow_launches = 0;
        c->graph_launches = c->graph_records = 0;
        QueryLayout L;
        upload_queries(c, queries, nq, strands, ix->sd.span, L);
        // --- seeds + X-drop (fused) --------------------------------------------------
        const double t1 = now_ms();
        int64_t nch = (int64_t)L.chunks.size();
        int64_t nraw = 0;
        if (nch > 0 && o.filter == SFE_FILTER_YDROP) {
            // the 2-D filter: both gapped halves of every seed hit around its middle column,
            // pruned at the X-drop value; a hit whose total reaches hsp_thresh becomes an HSP
            // spanning its seed window
            sfe_hit *hd = nullptr;
            const int64_t nhit = seed_hits_device(c, ix, L, &hd);
            st.seed_hits = nhit;
            // every hit becomes one extension item of a single batch (host records per half)
            if (nhit > ((int64_t)1 << 27)) fail(SFE_ENOMEM, "more than 2^27 seed hits for the 2-D filter");
            std::vector<sfe_hit> hits((size_t)nhit);
            copy_out(c, hits.data(), hd, (size_t)nhit * sizeof(sfe_hit));
            sync(c);
            std::vector<int32_t> uo(2 * (size_t)std::max(nq, 1), -1);
            for (size_t u = 0; u < L.units.size(); u++) uo[2 * L.units[u].query_id + L.units[u].strand] = (int32_t)u;
            const uint32_t off = (uint32_t)(ix->sd.span - 1) / 2;
            std::vector<ExtItem> fit((size_t)nhit);
            for (int64_t x = 0; x < nhit; x++)
                fit[x] = ExtItem{hits[x].t + off, hits[x].q + off, uo[2 * hits[x].query_id + hits[x].strand], 0};
            ScoreDesc fsc = sc;
            fsc.ydrop = sc.xdrop;
            fsc.gapped_thresh = sc.hsp_thresh;
            BatchResult fb;
            run_batch(c, ix, fit, fsc, cpl, SFE_SCHED_PLAIN, fb);
            std::vector<sfe_hsp> pass;
            for (int64_t x = 0; x < nhit; x++) {
                st.xdrop_columns += (int64_t)fb.alns[x].cells;
                if (fb.alns[x].score >= sc.hsp_thresh)
                    pass.push_back(sfe_hsp{hits[x].t, hits[x].q, (uint32_t)ix->sd.span, fb.alns[x].score,
                                           hits[x].query_id, hits[x].strand, {0, 0, 0}});
            }
            nraw = (int64_t)pass.size();
            sfe_hsp *raw = (sfe_hsp *)c->hsp_raw.ensure((size_t)std::max<int64_t>(nraw, 1) * sizeof(sfe_hsp));
            copy_in(c, raw, pass.data(), (size_t)nraw * sizeof(sfe_hsp));
            sync(c);
        } else if (nch > 0) {
            // room for one passing segment per 8 query bases (both strands) from the start: a launch
            // whose segments do not fit is run again with room for all of them
            uint64_t qbases = 0;
            for (const UnitDesc &ud : L.units) qbases += (uint64_t)ud.len;
            uint64_t capraw = std::max<uint64_t>(std::max<uint64_t>(c->hsp_raw.n / sizeof(sfe_hsp), 1u << 23),
                                                 qbases / 8);
            for (;;) {
                sfe_hsp *raw = (sfe_hsp *)c->hsp_raw.ensure(capraw * sizeof(sfe_hsp));
                unsigned long long *cnt = c->counters.as<unsigned long long>();
                HIPCHK(hipMemsetAsync(cnt, 0, 32, c->stream));
                HIPCHK(hipEventRecord(c->ev0, c->stream));
                launch_seed_xdrop(c->units_d.as<UnitDesc>(), c->chunks_d.as<Chunk>(), nch, ix->target.view(), 0, ix->nt,
                                  c->qplus.view(), c->qminus.view(), ix->offsets.as<uint32_t>(), ix->pos.as<uint32_t>(),
                                  ix->sd, sc, raw, capraw, cnt, c->stream);
                HIPCHK(hipGetLastError());
                HIPCHK(hipEventRecord(c->ev1, c->stream));
                unsigned long long hc[4];
                HIPCHK(hipMemcpyAsync(hc, cnt, 32, hipMemcpyDeviceToHost, c->stream));
                sync(c);
                if (hc[3]) fail(SFE_ERANGE, "an ungapped score reached 2^29");
                c->sx_ms += event_ms(c);
                c->sx_launches++;
                st.seed_hits = (int64_t)hc[0];
                nraw = (int64_t)hc[1];
                st.xdrop_columns = (int64_t)hc[2];
                if ((uint64_t)nraw <= capraw) break;
                capraw = (uint64_t)nraw + nraw / 8 + 1024;
            }
        }
        st.hsps_raw = nraw;
        const double t2 = now_ms();
        if (getenv("SFE_PROGRESS"))
            fprintf(stderr, "[sfe] seeds + x-drop: %lld hits, %lld passing, %.1f ms\n", (long long)st.seed_hits,
                    (long long)nraw, t2 - t1);
        int64_t nh = hsp_set(c, c->hsp_raw.as<sfe_hsp>(), nraw);
        st.hsps = nh;
        std::vector<sfe_hsp> hs((size_t)nh);
        copy_out(c, hs.data(), c->hsp_sorted.p, (size_t)nh * sizeof(sfe_hsp));
        sync(c);
        // --- cost model: predicted size of every HSP's two halves ----------------------
        std::vector<float> pred;
        const bool learned = o.model && o.schedule != SFE_SCHED_PLAIN && nh > 0;
        if (o.model && o.model->ctx->device != c->device) fail(SFE_EINVAL, "model lives on another device");
        if (learned) {
            const double tp = now_ms();
            float *F = (float *)c->feat_out.ensure((size_t)nh * SFE_MLP_NFEAT * 4);
            float *Y = (float *)c->feat_pred.ensure((size_t)nh * SFE_MLP_NOUT * 4);
            compute_features(c, ix, L, nq, c->hsp_sorted.as<sfe_hsp>(), nh, F);
            launch_mlp_forward(F, nh, o.model->p16.as<uint16_t>(), Y, c->stream);
            HIPCHK(hipGetLastError());
            pred.resize((size_t)nh * SFE_MLP_NOUT);
            copy_out(c, pred.data(), Y, pred.size() * 4);
            sync(c);
            st.ms_predict = now_ms() - tp;
        }
        std::vector<float> cost, extent;
        const double t3 = now_ms();
        // --- Alg. 3 rounds ------------------------------------------------------------
        std::vector<int32_t> unit_of(2 * (size_t)std::max(nq, 1), -1);
        for (size_t u = 0; u < L.units.size(); u++) unit_of[2 * L.units[u].query_id + L.units[u].strand] = (int32_t)u;
        const size_t NU = L.units.size();
        std::vector<std::vector<int64_t>> per_unit(NU);
        for (int64_t x = 0; x < nh; x++) per_unit[unit_of[2 * hs[x].query_id + hs[x].strand]].push_back(x);
        // per HSP state: 0 unresolved, 1 skipped (contained), 2 extension pending, 3 resolved, 4 in this batch
        std::vector<std::vector<uint8_t>> state(NU);
        // extension of each position once computed: alignment, batch whose edit runs hold its ops
        std::vector<std::vector<sfe_aln>> ext(NU);
        std::vector<std::vector<uint32_t>> ext_batch(NU);
        std::vector<OpsVec> batch_ops;                          // edit runs of every batch so far
        std::vector<std::vector<size_t>> open(NU);               // positions in state 0, ascending
        std::vector<UnitPaths> paths(NU);
        // deferral rule: a waiting extension is "doomed" when it will most likely be skipped at
        // commit (`perm`: its anchor lies in a committed alignment, for good); `wait` of an open
        // HSP: 1 its anchor lies on the path of an earlier waiting extension that is not
        // doomed, 2 in a committed alignment (skipped for good), 0 neither
        std::vector<std::vector<uint8_t>> doom_val(NU), doom_perm(NU), wait(NU);
        for (size_t u = 0; u < NU; u++) {
            const size_t n = per_unit[u].size();
            state[u].assign(n, 0);
            open[u].resize(n);
            for (size_t p = 0; p < n; p++) open[u][p] = p;
            ext[u].resize(n);
            ext_batch[u].assign(n, 0);
            paths[u].reset(ix->nt, n);
            doom_val[u].assign(n, 0);
            doom_perm[u].assign(n, 0);
            wait[u].assign(n, 0);
        }
        std::vector<size_t> cursor(NU, 0);
        std::vector<BoxGrid> boxes(NU);
        if (o.policy == SFE_POLICY_DEFER)
            for (size_t u = 0; u < NU; u++) boxes[u].reset(ix->nt);
        std::vector<sfe_aln> committed;
        std::vector<uint32_t> cbatch;           // per committed alignment: the batch holding its ops
        std::vector<ExtItem> items;
        std::vector<std::pair<int32_t, size_t>> item_ref;
        BatchResult br;
        const bool defer = o.policy == SFE_POLICY_DEFER;
        const bool progress = getenv("SFE_PROGRESS") != nullptr;
        const int64_t DB = o.near_band;                              // diagonal band of the nearness rule (< 0: off)
        auto anchor_of = [&](const sfe_hsp &h, uint32_t &ta, uint32_t &qa) {
            uint32_t off = (h.len - 1) / 2;
            ta = h.t0 + off;
            qa = h.q0 + off;
        };
        double host_ms = 0, book_ms = 0, commit_ms = 0;
        double ph[6] = {0, 0, 0, 0, 0, 0};      // doomed, pre-pass, unit scans, run writes, unit updates, commit
        std::vector<std::vector<uint16_t>> why(progress ? NU : 0);   // deferrals by path (lo byte) and nearness (hi)
        for (size_t u = 0; u < why.size(); u++) why[u].assign(per_unit[u].size(), 0);
        // nearness rule: diagonals taken, one bit set per host thread (cleared after each unit)
        std::vector<std::vector<uint64_t>> near_bits_t(16);
        std::vector<std::vector<size_t>> near_touched_t(16);
        std::vector<std::vector<ExtItem>> items_u(NU);
        std::vector<std::vector<size_t>> ref_u(NU);
        std::vector<std::vector<sfe_aln>> committed_u(NU);
        std::vector<std::vector<uint32_t>> cbatch_u(NU);
        std::vector<int64_t> shadow_u(NU, 0);
        std::vector<size_t> item_lo(NU + 1, 0);
        for (;;) {
            const double th = now_ms();
            items.clear();
            item_ref.clear();
            double tp = th;
            auto lap = [&](int k) { const double n = now_ms(); ph[k] += n - tp; tp = n; };
            if (defer) {
                // doomed flags of the waiting extensions in walking order: the anchor of waiting
                // extension p lies in a committed alignment, or on the path of an earlier waiting
                // extension that is not doomed itself (the rule only steers scheduling)
                // first, in parallel over pieces of the units: `perm`, and the earlier waiting
                // extensions whose paths hold each anchor; then each unit in order
                std::vector<std::pair<size_t, size_t>> jobs;
                for (size_t u = 0; u < NU; u++)
                    for (size_t a = 0; a < state[u].size(); a += 8192) jobs.push_back({u, a});
                std::vector<std::vector<std::pair<uint32_t, uint32_t>>> cand(jobs.size());   // (p, o)
                for_each_unit(jobs.size(), [&](size_t j, size_t) {
                    const size_t u = jobs[j].first;
                    const auto &stt = state[u];
                    const size_t end = std::min(stt.size(), jobs[j].second + 8192);
                    for (size_t p = jobs[j].second; p < end; p++) {
                        if (stt[p] != 2) continue;
                        const sfe_aln &a = ext[u][p];
                        if (!doom_perm[u][p] && paths[u].in_committed(a.anchor_t, a.anchor_q)) doom_perm[u][p] = 1;
                        if (doom_perm[u][p]) continue;
                        paths[u].set.search(a.anchor_t, a.anchor_q, [&](size_t o) { return o < p && stt[o] == 2; },
                                            [&](size_t o) {
                                                cand[j].push_back({(uint32_t)p, (uint32_t)o});
                                                return false;
                                            });
                    }
                });
                for_each_unit(NU, [&](size_t u, size_t) {
                    const auto &stt = state[u];
                    auto &dv = doom_val[u];
                    for (size_t p = 0; p < stt.size(); p++)
                        if (stt[p] == 2) dv[p] = doom_perm[u][p];
                    for (size_t j = 0; j < jobs.size(); j++) {
                        if (jobs[j].first != u) continue;
                        for (const auto &po : cand[j])
                            if (!dv[po.first] && dv[po.second] == 0) dv[po.first] = 2;    // 2: doomed by a path
                    }
                });
            }
            lap(0);
            {
                // anchors already on an M column of a committed alignment stay skipped for good:
                // found for every open HSP first, in parallel over pieces of the open lists
                std::vector<std::pair<size_t, size_t>> jobs;
                for (size_t u = 0; u < NU; u++)
                    for (size_t a = 0; a < open[u].size(); a += 8192) jobs.push_back({u, a});
                for_each_unit(jobs.size(), [&](size_t j, size_t) {
                    const size_t u = jobs[j].first;
                    const size_t end = std::min(open[u].size(), jobs[j].second + 8192);
                    const auto &stt = state[u];
                    const auto &dv = doom_val[u];
                    for (size_t q = jobs[j].second; q < end; q++) {
                        const size_t p = open[u][q];
                        if (stt[p] != 0) continue;
                        uint32_t ta, qa;
                        anchor_of(hs[per_unit[u][p]], ta, qa);
                        if (paths[u].in_committed(ta, qa)) {
                            wait[u][p] = 2;
                        } else if (defer) {
                            // on the path of an earlier extension that may still commit
                            wait[u][p] = paths[u].set.contains(ta, qa, [&](size_t o) { return o < p && stt[o] == 2; },
                                                               [&](size_t o) { return dv[o] == 0; });
                        }
                    }
                });
                for_each_unit(NU, [&](size_t u, size_t) {
                    for (size_t p : open[u])
                        if (wait[u][p] == 2) state[u][p] = 1;
                });
            }
            lap(1);
            for_each_unit(NU, [&](size_t u, size_t tix) {        // Alg. 3 batch gathering, per unit
                auto &near_bits = near_bits_t[tix];
                auto &near_touched = near_touched_t[tix];
                auto &uitems = items_u[u];
                auto &uref = ref_u[u];
                uitems.clear();
                uref.clear();
                auto &lst = per_unit[u];
                auto &stt = state[u];
                int64_t taken = 0;
                // diagonals of the HSPs this batch has taken so far in the unit (bit d + qlen)
                const int64_t qlen = L.units[u].len;
                const size_t nwords = (size_t)((ix->nt + qlen + std::max<int64_t>(DB, 0) + 1) / 64 + 2);
                if (near_bits.size() < nwords) near_bits.resize(nwords, 0);
                std::vector<size_t> still;
                still.reserve(open[u].size());
                size_t q = 0;
                for (; q < open[u].size() && taken < K; q++) {
                    const size_t p = open[u][q];
                    if (stt[p] != 0) continue;
                    uint32_t ta, qa;
                    anchor_of(hs[lst[p]], ta, qa);
                    if (defer) {
                        // on the path of an earlier extension that may still commit: wait for it
                        if (wait[u][p] == 1) {
                            if (progress) why[u][p] += 1;
                            still.push_back(p);
                            continue;
                        }
                        // inside a committed alignment but off its path: such HSPs are extended
                        // side by side (each may start a separate alignment of the region)
                        if (DB > 0) {
                            const int64_t x = (int64_t)ta - (int64_t)qa + qlen;
                            const int64_t lo = std::max<int64_t>(0, x - DB), hi = x + DB;
                            bool close = false;
                            for (int64_t w = lo >> 6; w <= (hi >> 6) && !close; w++) {
                                uint64_t m = near_bits[(size_t)w];
                                if (w == (lo >> 6)) m &= ~0ull << (lo & 63);
                                if (w == (hi >> 6)) m &= (hi & 63) == 63 ? ~0ull : ((2ull << (hi & 63)) - 1);
                                close = m != 0;
                            }
                            if (close && !boxes[u].inside(ta, qa)) {                      // likely the same region
                                if (progress) why[u][p] += 256;
                                still.push_back(p);
                                continue;
                            }
                            uint64_t &word = near_bits[(size_t)(x >> 6)];
                            if (!word) near_touched.push_back((size_t)(x >> 6));
                            word |= 1ull << (x & 63);
                        }
                    }
                    uitems.push_back(ExtItem{ta, qa, (int32_t)u, 0});
                    uref.push_back(p);
                    stt[p] = 4;
                    taken++;
                }
                for (; q < open[u].size(); q++)
                    if (stt[open[u][q]] == 0) still.push_back(open[u][q]);
                open[u].swap(still);
                for (size_t w : near_touched) near_bits[w] = 0;
                near_touched.clear();
            });
            for (size_t u = 0; u < NU; u++) {                      // the batch in unit order
                item_lo[u] = items.size();
                items.insert(items.end(), items_u[u].begin(), items_u[u].end());
                for (size_t p : ref_u[u]) item_ref.push_back({(int32_t)u, p});
            }
            item_lo[NU] = items.size();
            lap(2);
            const double scan_round_ms = now_ms() - th;
            host_ms += scan_round_ms;
            if (items.empty()) break;
            st.rounds++;
            const double tr = now_ms();
            if (learned) {
                cost.resize(2 * items.size());
                extent.resize(2 * items.size());
                for (size_t x = 0; x < items.size(); x++) {
                    const int64_t hx = per_unit[item_ref[x].first][item_ref[x].second];
                    cost[2 * x] = pred[(size_t)hx * 4 + 0];
                    extent[2 * x] = pred[(size_t)hx * 4 + 1];
                    cost[2 * x + 1] = pred[(size_t)hx * 4 + 2];
                    extent[2 * x + 1] = pred[(size_t)hx * 4 + 3];
                }
            }
            run_batch(c, ix, items, sc, cpl, o.schedule, br, learned ? &cost : nullptr,
                      learned ? &extent : nullptr);                                   // the batch on the GPU
            st.predicted_halves += br.predicted;
            st.mispredicted_halves += br.mispredicted;
            if (progress) {
                fprintf(stderr, "[sfe] batch %lld: %zu extensions, %.1f ms (scan %.1f ms), %zu committed so far\n",
                        (long long)st.rounds, items.size(), now_ms() - tr, scan_round_ms,
                        [&] { size_t n = 0; for (auto &v : committed_u) n += v.size(); return n; }());
                size_t xl = 0;
                int64_t kl = -1, nlong = 0;
                for (size_t x = 0; x < items.size(); x++)
                    for (int s2 = 0; s2 < 2; s2++) {
                        const int64_t kk = br.halves[2 * x + s2].k_last;
                        if (kk > 100000) nlong++;
                        if (kk > kl) { kl = kk; xl = x; }
                    }
                if (kl >= 0) {
                    const int32_t u = item_ref[xl].first;
                    const size_t p = item_ref[xl].second;
                    const sfe_hsp &h = hs[per_unit[u][p]];
                    fprintf(stderr, "[sfe]   longest half %lld antidiagonals (item unit %d pos %zu of %zu, score %d, "
                                    "diag %lld, deferred %d by path, %d by nearness); %lld halves > 100k\n",
                            (long long)kl, u, p, per_unit[u].size(), (int)h.score, (long long)h.t0 - (long long)h.q0,
                            why[u][p] & 255, why[u][p] >> 8, (long long)nlong);
                }
            }
            const double th2 = now_ms();
            tp = th2;
            st.overflow_reruns += br.reruns;
            st.extensions += (int64_t)items.size();
            const uint32_t bno = (uint32_t)batch_ops.size();
            batch_ops.push_back(std::move(br.ops));
            br.ops = OpsVec();
            const uint32_t *bops = batch_ops.back().data();
            for (size_t x = 0; x < items.size(); x++) st.cells += (int64_t)br.alns[x].cells;
            {
                // M runs of the passing extensions: counted and written in parallel over pieces
                // of the batch, each unit's at the end of its store
                const size_t nb = items.size();
                const size_t piece = 4096;
                std::vector<uint32_t> nrun(nb, 0);
                std::vector<size_t> roff(nb, 0);
                for_each_unit((nb + piece - 1) / piece, [&](size_t j, size_t) {
                    for (size_t x = j * piece; x < std::min(nb, (j + 1) * piece); x++)
                        if (br.alns[x].flags & SFE_ALN_PASSED)
                            nrun[x] = PathSet::count_runs(br.alns[x], bops + br.alns[x].ops_offset);
                });
                for (size_t u = 0; u < NU; u++) {
                    size_t at = paths[u].runs.n;
                    for (size_t x = item_lo[u]; x < item_lo[u + 1]; x++) {
                        roff[x] = at;
                        at += nrun[x];
                    }
                    paths[u].runs.grow(at - paths[u].runs.n);
                    paths[u].runs.n = at;
                }
                std::vector<int32_t> unit_x(nb);
                for (size_t u = 0; u < NU; u++)
                    for (size_t x = item_lo[u]; x < item_lo[u + 1]; x++) unit_x[x] = (int32_t)u;
                for_each_unit((nb + piece - 1) / piece, [&](size_t j, size_t) {
                    for (size_t x = j * piece; x < std::min(nb, (j + 1) * piece); x++)
                        if (nrun[x])
                            PathSet::write_runs(paths[unit_x[x]].runs, roff[x], br.alns[x], bops + br.alns[x].ops_offset);
                });
                lap(3);
                for_each_unit(NU, [&](size_t u, size_t) {
                    for (size_t x = item_lo[u]; x < item_lo[u + 1]; x++) {
                        const sfe_aln &a = br.alns[x];
                        const size_t p = item_ref[x].second;
                        ext[u][p] = a;
                        ext_batch[u][p] = bno;
                        if (a.flags & SFE_ALN_PASSED) {
                            paths[u].add(a, roff[x], nrun[x], p);
                            if (defer) boxes[u].add(a);
                        }
                        state[u][p] = 2;
                    }
                });
            }
            lap(4);
            const double th3 = now_ms();
            book_ms += th3 - th2;
            for_each_unit(NU, [&](size_t u, size_t) {             // in-order commit (Alg. 1 decisions)
                auto &lst = per_unit[u];
                auto &stt = state[u];
                size_t &cur = cursor[u];
                while (cur < lst.size()) {
                    const size_t p = cur;
                    if (stt[p] == 1 || stt[p] == 3) { cur++; continue; }
                    if (stt[p] == 2) {
                        const sfe_aln &a = ext[u][p];
                        if (paths[u].in_committed(a.anchor_t, a.anchor_q)) {
                            shadow_u[u]++;
                        } else if (a.flags & SFE_ALN_PASSED) {
                            // ops stay in their batch's buffer until the output is written
                            paths[u].commit(a, p);
                            committed_u[u].push_back(a);
                            cbatch_u[u].push_back(ext_batch[u][p]);
                        }
                        stt[p] = 3;
                        cur++;
                        continue;
                    }
                    uint32_t ta, qa;
                    anchor_of(hs[lst[p]], ta, qa);
                    if (paths[u].in_committed(ta, qa)) { stt[p] = 1; cur++; continue; }
                    break;                                          // needs an extension first
                }
            });
            lap(5);
            commit_ms += now_ms() - th3;
            host_ms += now_ms() - th2;
        }
        if (progress) {
            fprintf(stderr, "[sfe] host scan/commit time %.1f ms (scan %.1f, bookkeeping %.1f, commit %.1f)\n", host_ms,
                    host_ms - book_ms - commit_ms, book_ms, commit_ms);
            fprintf(stderr, "[sfe]   phases: doomed %.1f, pre-pass %.1f, unit scans %.1f, run writes %.1f, unit updates "
                    "%.1f, commit %.1f ms\n", ph[0], ph[1], ph[2], ph[3], ph[4], ph[5]);
            for (size_t u = 0; u < NU; u++)
                fprintf(stderr, "[sfe]   unit %zu: %zu HSPs, %zu extension paths (%zu M runs), %zu committed\n", u,
                        per_unit[u].size(), paths[u].set.paths.size(), paths[u].runs.n,
                        paths[u].done.paths.size());
        }
        for (size_t u = 0; u < NU; u++) {
            if (cursor[u] != per_unit[u].size()) fail(SFE_EINTERNAL, "commit did not finish");
            committed.insert(committed.end(), committed_u[u].begin(), committed_u[u].end());
            cbatch.insert(cbatch.end(), cbatch_u[u].begin(), cbatch_u[u].end());
            st.shadow += shadow_u[u];
        }
        st.committed = (int64_t)committed.size();
        const double t4 = now_ms();
        // --- output in (query, strand, t_start, q_start, t_end, q_end, anchor) order ---
        std::vector<int64_t> order(committed.size());
        for (size_t x = 0; x < order.size(); x++) order[x] = (int64_t)x;
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
            const sfe_aln &x = committed[a], &y = committed[b];
            auto kx = std::make_tuple(x.query_id, x.strand, x.t_start, x.q_start, x.t_end, x.q_end, x.anchor_t, x.anchor_q);
            auto ky = std::make_tuple(y.query_id, y.strand, y.t_start, y.q_start, y.t_end, y.q_end, y.anchor_t, y.anchor_q);
            return kx < ky;
        });
        uint64_t total_ops = 0;
        for (const sfe_aln &a : committed) total_ops += a.ops_len;
        *n_alns = (int64_t)committed.size();
        *n_ops = (int64_t)total_ops;
        if (stats) {
            st.ms_seed_xdrop = t2 - t1;
            st.ms_hsp_set = t3 - t2;
            st.ms_extend = t4 - t3;
            st.ms_total = now_ms() - t0;
            st.ydrop_launches = c->ydrop_launches;
            st.narrow_launches = c->narrow_launches;
            st.graph_launches = c->graph_launches;
            st.graph_records = c->graph_records;
            st.ydrop_kernel_cells = c->ydrop_cells;
            st.seed_xdrop_launches = c->sx_launches;
            st.ms_ydrop_kernel = c->ydrop_ms;
            st.ms_seed_xdrop_kernel = c->sx_ms;
            *stats = st;
        }
        if (*n_alns > cap || *n_ops > ops_cap) fail(SFE_ECAPACITY, "alignment or ops buffer too small");
        if ((*n_alns && !out) || (*n_ops && !ops)) fail(SFE_EINVAL, "null output");
        std::vector<sfe_aln> oa(committed.size());
        OpsVec oo(total_ops);
        uint64_t at = 0;
        for (size_t x = 0; x < order.size(); x++) {
            oa[x] = committed[order[x]];
            oa[x].ops_offset = at;
            at += oa[x].ops_len;
        }
        // edit runs straight from the batch buffers, in parallel over pieces of the output
        const size_t piece = 4096;
        for_each_unit((order.size() + piece - 1) / piece, [&](size_t j, size_t) {
            for (size_t x = j * piece; x < std::min(order.size(), (j + 1) * piece); x++) {
                const sfe_aln &a = committed[order[x]];
                const uint32_t *src = batch_ops[cbatch[order[x]]].data() + a.ops_offset;
                std::copy(src, src + a.ops_len, oo.begin() + (ptrdiff_t)oa[x].ops_offset);
            }
        });
        copy_out(c, out, oa.data(), oa.size() * sizeof(sfe_aln));
        copy_out(c, ops, oo.data(), oo.size() * 4);
        sync(c);
        if (stats) stats->ms_total = now_ms() - t0;
    });
}

sfe_status sfe_ctx_set_tuning(sfe_ctx *c, const sfe_tuning *t) {
    if (!c || !t || t->wave_group_cap < 0 || t->use_graphs < 0 || t->use_graphs > 1 || t->wide_scores < 0 ||
        t->wide_scores > 1 || t->persist_waves_per_cu < 0 || t->persist_waves_per_cu > 64 || t->adaptive_halves < 0)
        return SFE_EINVAL;
    c->tuning = *t;
    return SFE_OK;
}

sfe_status sfe_autotune(sfe_ctx *c, const sfe_index *ix, const sfe_seq *queries, int32_t nq, const sfe_scoring *scp,
                        int64_t sample_bases, sfe_align_opts *opts, sfe_tune_report *report) {
    if (!c || !ix || !opts || nq < 1 || !queries || sample_bases < 1) return SFE_EINVAL;
    std::vector<sfe_seq> sample((size_t)nq);
    for (int32_t i = 0; i < nq; i++) {
        sample[i] = queries[i];
        sample[i].length = std::min<int64_t>(queries[i].length, sample_bases);
    }
    const sfe_tuning saved = c->tuning;
    sfe_tune_report rep{};
    double best_ms = 1e300;
    sfe_align_opts best = *opts;
    int32_t best_cap = saved.wave_group_cap;
    std::vector<sfe_aln> out(1 << 16);
    std::vector<uint32_t> ops(1 << 22);
    const int cpls[2] = {4, 6};
    const int caps[2] = {0, 8192};
    const int wpcs[2] = {8, 16};
    // with a cost model only the schedules that use it compete
    const int sched_lo = opts->model ? SFE_SCHED_PERSISTENT : SFE_SCHED_PLAIN;
    bool first = true;
    int32_t best_wpc = saved.persist_waves_per_cu;
    for (int cap : caps)
        for (int sched = sched_lo; sched <= SFE_SCHED_BINNED; sched++)
            for (int wpc : wpcs)
            for (int cpl : cpls) {
                // plain and binned launches have no grid knob
                if ((sched == SFE_SCHED_PLAIN || sched == SFE_SCHED_BINNED) && wpc != wpcs[0]) continue;
                sfe_align_opts o = *opts;
                o.max_cells_per_lane = cpl;
                o.schedule = sched;
                if (sched == SFE_SCHED_PLAIN) o.model = nullptr;
                c->tuning.wave_group_cap = cap;
                c->tuning.persist_waves_per_cu =
                    (sched == SFE_SCHED_PLAIN || sched == SFE_SCHED_BINNED) ? saved.persist_waves_per_cu : wpc;
                sfe_stats st{};
                int64_t na = 0, no = 0;
                sfe_status r = SFE_OK;
                double ms = 1e300;
                // three timed runs (the fastest counts); the very first candidate warms up once more
                for (int rep_i = first ? 4 : 3; rep_i > 0; rep_i--) {
                    for (;;) {
                        r = sfe_align(c, ix, sample.data(), nq, scp, &o, out.data(), (int64_t)out.size(), &na,
                                      ops.data(), (int64_t)ops.size(), &no, &st);
                        if (r == SFE_ECAPACITY && (na > (int64_t)out.size() || no > (int64_t)ops.size())) {
                            out.resize(std::max<size_t>(out.size(), (size_t)na));
                            ops.resize(std::max<size_t>(ops.size(), (size_t)no));
                            continue;
                        }
                        break;
                    }
                    if (r != SFE_OK) break;
                    if (!(first && rep_i == 4)) ms = std::min(ms, st.ms_extend);
                }
                first = false;
                if (r != SFE_OK) {
                    c->tuning = saved;
                    return r;
                }
                if (rep.n < 32) rep.entries[rep.n++] = sfe_tune_entry{cpl, sched, cap, c->tuning.persist_waves_per_cu, ms};
                if (ms < best_ms) {
                    best_ms = ms;
                    best = o;
                    best_cap = cap;
                    best_wpc = c->tuning.persist_waves_per_cu;
                    rep.best = rep.n - 1;
                }
            }
    c->tuning = saved;
    c->tuning.wave_group_cap = best_cap;
    c->tuning.persist_waves_per_cu = best_wpc;
    opts->max_cells_per_lane = best.max_cells_per_lane;
    opts->schedule = best.schedule;
    if (report) *report = rep;
    return SFE_OK;
}

sfe_status sfe_ctx_get_tuning(const sfe_ctx *c, sfe_tuning *t) {
    if (!c || !t) return SFE_EINVAL;
    *t = c->tuning;
    return SFE_OK;
}

sfe_status sfe_hsp_features(sfe_ctx *c, const sfe_index *ix, const sfe_seq *queries, int32_t nq, const sfe_hsp *hsps,
                            int64_t n, float *features) {
    if (!c || !ix || n < 0) return SFE_EINVAL;
    return guard(c, [&] {
        QueryLayout L;
        upload_queries(c, queries, nq, 3, ix->sd.span, L);
        if (n == 0) return;
        if (!features) fail(SFE_EINVAL, "null features");
        std::vector<sfe_hsp> hh = checked_hsps(c, ix, queries, nq, hsps, n);
        sfe_hsp *hd = (sfe_hsp *)c->feat_hsp.ensure((size_t)n * sizeof(sfe_hsp));
        copy_in(c, hd, hh.data(), (size_t)n * sizeof(sfe_hsp));
        float *F = (float *)c->feat_out.ensure((size_t)n * SFE_MLP_NFEAT * 4);
        compute_features(c, ix, L, nq, hd, n, F);
        copy_out(c, features, F, (size_t)n * SFE_MLP_NFEAT * 4);
        sync(c);
    });
}

sfe_status sfe_extension_log(sfe_ctx *c, const sfe_index *ix, const sfe_seq *queries, int32_t nq, const sfe_hsp *hsps,
                             int64_t n, const sfe_scoring *scp, float *features, float *targets) {
    if (!c || !ix || n < 0) return SFE_EINVAL;
    return guard(c, [&] {
        ScoreDesc sc = check_scoring(scp);
        QueryLayout L;
        upload_queries(c, queries, nq, 3, ix->sd.span, L);
        if (n == 0) return;
        if (!features || !targets) fail(SFE_EINVAL, "null output");
        std::vector<sfe_hsp> hh = checked_hsps(c, ix, queries, nq, hsps, n);
        std::vector<ExtItem> items((size_t)n);
        for (int64_t x = 0; x < n; x++) {
            const sfe_hsp &h = hh[x];
            const uint32_t off = (h.len - 1) / 2;
            items[x] = ExtItem{h.t0 + off, h.q0 + off, (int32_t)(2 * h.query_id + h.strand), 0};
        }
        BatchResult br;
        run_batch(c, ix, items, sc, 6, SFE_SCHED_PLAIN, br);
        std::vector<float> tg((size_t)n * SFE_MLP_NOUT);
        for (int64_t x = 0; x < n; x++)
            for (int s = 0; s < 2; s++) {
                const HalfResult &r = br.halves[2 * x + s];
                tg[x * 4 + 2 * s] = (float)std::log2(1.0 + (double)r.cells);
                tg[x * 4 + 2 * s + 1] = (float)std::log2(1.0 + (double)r.i_end + (double)r.j_end);
            }
        sfe_hsp *hd = (sfe_hsp *)c->feat_hsp.ensure((size_t)n * sizeof(sfe_hsp));
        copy_in(c, hd, hh.data(), (size_t)n * sizeof(sfe_hsp));
        float *F = (float *)c->feat_out.ensure((size_t)n * SFE_MLP_NFEAT * 4);
        compute_features(c, ix, L, nq, hd, n, F);
        copy_out(c, features, F, (size_t)n * SFE_MLP_NFEAT * 4);
        copy_out(c, targets, tg.data(), tg.size() * 4);
        sync(c);
    });
}

sfe_status sfe_model_create(sfe_ctx *c, const float *params, sfe_model **out) {
    if (!c || !params || !out) return SFE_EINVAL;
    *out = nullptr;
    sfe_model *m = new (std::nothrow) sfe_model;
    if (!m) return SFE_ENOMEM;
    m->ctx = c;
    m->device = c->device;
    sfe_status st = guard(c, [&] {
        const size_t NP = SFE_MLP_NPARAMS;
        m->master.ensure(NP * 4);
        m->m.ensure(NP * 4);
        m->v.ensure(NP * 4);
        m->p16.ensure(NP * 2);
        HIPCHK(hipMemcpyAsync(m->master.p, params, NP * 4, hipMemcpyDefault, c->stream));
        HIPCHK(hipMemsetAsync(m->m.p, 0, NP * 4, c->stream));
        HIPCHK(hipMemsetAsync(m->v.p, 0, NP * 4, c->stream));
        launch_mlp_round(m->master.as<float>(), m->p16.as<uint16_t>(), c->stream);
        HIPCHK(hipGetLastError());
        sync(c);
    });
    if (st != SFE_OK) {
        delete m;
        return st;
    }
    *out = m;
    return SFE_OK;
}

void sfe_model_destroy(sfe_model *m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    delete m;                           // hipFree waits for work that still uses the buffers
    (void)hipGetLastError();
}

sfe_status sfe_model_params(const sfe_model *m, float *params) {
    if (!m || !params) return SFE_EINVAL;
    sfe_ctx *c = m->ctx;
    return guard(c, [&] {
        copy_out(c, params, m->master.p, (size_t)SFE_MLP_NPARAMS * 4);
        sync(c);
    });
}

sfe_status sfe_model_predict(sfe_model *m, const float *x, int64_t n, float *y) {
    if (!m || n < 0) return SFE_EINVAL;
    sfe_ctx *c = m->ctx;
    return guard(c, [&] {
        if (n == 0) return;
        if (!x || !y) fail(SFE_EINVAL, "null input or output");
        float *xd = (float *)m->x.ensure((size_t)n * SFE_MLP_NFEAT * 4);
        float *yd = (float *)m->y.ensure((size_t)n * SFE_MLP_NOUT * 4);
        copy_in(c, xd, x, (size_t)n * SFE_MLP_NFEAT * 4);
        launch_mlp_forward(xd, n, m->p16.as<uint16_t>(), yd, c->stream);
        HIPCHK(hipGetLastError());
        copy_out(c, y, yd, (size_t)n * SFE_MLP_NOUT * 4);
        sync(c);
    });
}

sfe_status sfe_model_grad(sfe_model *m, const float *x, const float *t, int64_t n, float *grad, float *loss) {
    if (!m || n < 1 || n > (int64_t)INT32_MAX - 64) return SFE_EINVAL;
    sfe_ctx *c = m->ctx;
    return guard(c, [&] {
        if (!x || !t || !grad) fail(SFE_EINVAL, "null argument");
        const size_t NP = SFE_MLP_NPARAMS;
        const int nb = (int)((n + 63) / 64);
        float *xd = (float *)m->x.ensure((size_t)n * SFE_MLP_NFEAT * 4);
        float *td = (float *)m->t.ensure((size_t)n * SFE_MLP_NOUT * 4);
        uint32_t *ids = (uint32_t *)m->ids.ensure((size_t)n * 4);
        float *part = (float *)m->part.ensure((size_t)nb * NP * 4);
        float *sse = (float *)m->sse.ensure((size_t)nb * 4);
        float *gd = (float *)m->grad.ensure(NP * 4);
        float *ld = (float *)m->loss.ensure(4);
        copy_in(c, xd, x, (size_t)n * SFE_MLP_NFEAT * 4);
        copy_in(c, td, t, (size_t)n * SFE_MLP_NOUT * 4);
        k_iota<<<grid(n, 256), 256, 0, c->stream>>>(ids, n);
        launch_mlp_grad(xd, td, (const int32_t *)ids, (int32_t)n, m->p16.as<uint16_t>(), part, sse, c->stream);
        launch_mlp_apply(part, nb, sse, (int32_t)n, gd, nullptr, nullptr, nullptr, nullptr, 0.f, 1.f, 1.f, ld,
                         c->stream);
        HIPCHK(hipGetLastError());
        copy_out(c, grad, gd, NP * 4);
        if (loss) copy_out(c, loss, ld, 4);
        sync(c);
    });
}

sfe_status sfe_model_grad_noalloc(sfe_model *m, const float *x, const float *t, int64_t n, float *grad,
                                  float *loss) {
    if (!m || n < 1) return SFE_EINVAL;
    sfe_ctx *c = m->ctx;
    return guard(c, [&] {
        if (n > SFE_NOALLOC_MAX_SAMPLES) fail(SFE_EINVAL, "more samples than the fixed working memory holds");
        if (!x || !t || !grad || !loss) fail(SFE_EINVAL, "null argument");
        if (!is_device_ptr(x) || !is_device_ptr(t) || !is_device_ptr(grad) || !is_device_ptr(loss))
            fail(SFE_EINVAL, "inputs and outputs must be device memory");
        uint8_t *base = scratch_of(c->device);
        if (!base) fail(SFE_EINTERNAL, "working memory of this device was not set up");
        uint32_t *ids = (uint32_t *)base;
        float *sse = (float *)(base + kScratchIds);
        float *part = (float *)(base + kScratchIds + kScratchSse);
        const int nb = (int)((n + 63) / 64);
        k_iota<<<grid(n, 256), 256, 0, c->stream>>>(ids, n);
        launch_mlp_grad(x, t, (const int32_t *)ids, (int32_t)n, m->p16.as<uint16_t>(), part, sse, c->stream);
        launch_mlp_apply(part, nb, sse, (int32_t)n, grad, nullptr, nullptr, nullptr, nullptr, 0.f, 1.f, 1.f, loss,
                         c->stream);
        HIPCHK(hipGetLastError());
    });
}

sfe_status sfe_model_train(sfe_model *m, const float *x, const float *t, int64_t n, const int32_t *order,
                           int64_t n_order, int32_t batch, float lr, float *losses) {
    if (!m || n < 1 || n_order < 0 || batch < 1 || batch > (1 << 20) || !(lr > 0.0f)) return SFE_EINVAL;
    sfe_ctx *c = m->ctx;
    return guard(c, [&] {
        if (n_order == 0) return;
        if (!x || !t || !order) fail(SFE_EINVAL, "null argument");
        std::vector<int32_t> ord((size_t)n_order);
        HIPCHK(hipMemcpyAsync(ord.data(), order, (size_t)n_order * 4, hipMemcpyDefault, c->stream));
        sync(c);
        for (int32_t id : ord)
            if (id < 0 || id >= n) fail(SFE_EINVAL, "sample id out of range");
        const size_t NP = SFE_MLP_NPARAMS;
        const int64_t steps = (n_order + batch - 1) / batch;
        const int nbmax = (batch + 63) / 64;
        float *xd = (float *)m->x.ensure((size_t)n * SFE_MLP_NFEAT * 4);
        float *td = (float *)m->t.ensure((size_t)n * SFE_MLP_NOUT * 4);
        int32_t *ids = (int32_t *)m->ids.ensure((size_t)n_order * 4);
        float *part = (float *)m->part.ensure((size_t)nbmax * NP * 4);
        float *sse = (float *)m->sse.ensure((size_t)nbmax * 4);
        float *ld = (float *)m->loss.ensure((size_t)steps * 4);
        copy_in(c, xd, x, (size_t)n * SFE_MLP_NFEAT * 4);
        copy_in(c, td, t, (size_t)n * SFE_MLP_NOUT * 4);
        copy_in(c, ids, ord.data(), (size_t)n_order * 4);
        const bool graph = c->tuning.use_graphs == 1;
        hipGraph_t g = nullptr;
        if (graph) HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        for (int64_t s = 0; s < steps; s++) {
            const int32_t B = (int32_t)std::min<int64_t>(batch, n_order - s * batch);
            const int nb = (B + 63) / 64;
            launch_mlp_grad(xd, td, ids + s * batch, B, m->p16.as<uint16_t>(), part, sse, c->stream);
            m->step++;
            const float c1 = (float)(1.0 - std::pow(0.9, (double)m->step));
            const float c2 = (float)(1.0 - std::pow(0.999, (double)m->step));
            launch_mlp_apply(part, nb, sse, B, nullptr, m->master.as<float>(), m->m.as<float>(), m->v.as<float>(),
                             m->p16.as<uint16_t>(), lr, c1, c2, ld + s, c->stream);
        }
        HIPCHK(hipGetLastError());
        if (graph) {
            // the whole step sequence as one graph, launched once
            HIPCHK(hipStreamEndCapture(c->stream, &g));
            hipGraphExec_t ge = nullptr;
            hipError_t e1 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            hipError_t e2 = e1 == hipSuccess ? hipGraphLaunch(ge, c->stream) : e1;
            hipError_t e3 = e2 == hipSuccess ? hipStreamSynchronize(c->stream) : e2;
            if (ge) (void)hipGraphExecDestroy(ge);
            (void)hipGraphDestroy(g);
            HIPCHK(e3);
        }
        if (losses) copy_out(c, losses, ld, (size_t)steps * 4);
        sync(c);
    });
}


sfe_status sfe_model_save(const sfe_model *m, const char *path) {
    if (!m || !path) return SFE_EINVAL;
    sfe_ctx *c = m->ctx;
    return guard(c, [&] {
        const size_t NP = SFE_MLP_NPARAMS;
        std::vector<uint8_t> buf(kModelBytes, 0);
        memcpy(buf.data(), kModelMagic, 8);
        const uint32_t hdr[4] = {1u, 1u, (uint32_t)NP, 0u};
        memcpy(buf.data() + 8, hdr, 16);
        memcpy(buf.data() + 24, &m->step, 8);
        uint8_t *body = buf.data() + kModelHeader;
        copy_out(c, body, m->master.p, NP * 4);
        copy_out(c, body + NP * 4, m->m.p, NP * 4);
        copy_out(c, body + 2 * NP * 4, m->v.p, NP * 4);
        sync(c);
        const uint64_t h = fnv1a(buf.data(), kModelBytes - 8);
        memcpy(buf.data() + kModelBytes - 8, &h, 8);
        FILE *f = fopen(path, "wb");
        if (!f) fail(SFE_EIO, std::string("cannot create ") + path);
        const size_t put = fwrite(buf.data(), 1, buf.size(), f);
        const bool bad = fclose(f) != 0 || put != buf.size();
        if (bad) fail(SFE_EIO, std::string("cannot write ") + path);
    });
}

sfe_status sfe_model_load(sfe_ctx *c, const char *path, sfe_model **out) {
    if (!path || (!c) != (!out)) return SFE_EINVAL;
    if (out) *out = nullptr;
    std::vector<uint8_t> buf;
    std::string why;
    const sfe_status st = read_model_file(path, buf, why);
    if (st != SFE_OK) {
        if (c) c->last_error = why;
        return st;
    }
    if (!c) return SFE_OK;             // check only
    const size_t NP = SFE_MLP_NPARAMS;
    const uint8_t *body = buf.data() + kModelHeader;
    std::vector<float> params(NP);
    memcpy(params.data(), body, NP * 4);
    sfe_model *m = nullptr;
    sfe_status r = sfe_model_create(c, params.data(), &m);
    if (r != SFE_OK) return r;
    r = guard(c, [&] {
        copy_in(c, m->m.p, body + NP * 4, NP * 4);
        copy_in(c, m->v.p, body + 2 * NP * 4, NP * 4);
        memcpy(&m->step, buf.data() + 24, 8);
        sync(c);
    });
    if (r != SFE_OK) {
        sfe_model_destroy(m);
        return r;
    }
    *out = m;
    return SFE_OK;
}

const char *sfe_status_str(sfe_status s) {
    switch (s) {
    case SFE_OK: return "ok";
    case SFE_EINVAL: return "invalid argument";
    case SFE_ENOMEM: return "out of memory";
    case SFE_ECAPACITY: return "output capacity too small";
    case SFE_ERANGE: return "value range exceeded";
    case SFE_EDEVICE: return "device error";
    case SFE_EINTERNAL: return "internal error";
    case SFE_EIO: return "file input/output failed";
    default: return "unknown status";
    }
}

const char *sfe_last_error(const sfe_ctx *c) { return c ? c->last_error.c_str() : "null context"; }

}  // extern "C"
