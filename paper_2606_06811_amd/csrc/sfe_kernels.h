// sfe_kernels.h -- kernel declarations and small device-side descriptors.
#pragma once
#include "sfe_internal.h"

namespace sfe {

struct ScoreDesc {
    int32_t sub[5][5];
    int32_t gap_open, gap_extend, xdrop, hsp_thresh, ydrop, gapped_thresh;
};

// One (query, strand) unit: its bases are [seq_start, seq_start + len) of the
// plus or minus query set.
struct UnitDesc {
    int64_t seq_start;
    int64_t len;
    int32_t query_id;
    int32_t strand;
};

// 64 consecutive query windows of one unit, starting at window w0.
struct Chunk {
    int32_t unit;
    int32_t w0;
};

struct QueryDesc {
    int64_t start;      // same start in the plus and the minus set
    int64_t len;
};

// A batch item of the gapped stage: anchor column (ta, qa) of a unit.
struct ExtItem {
    uint32_t ta, qa;
    int32_t unit;
    int32_t pad;
};

hipError_t upload_encoding_table(hipStream_t st);

__global__ void k_pack(const uint8_t *txt, int64_t len, int64_t out_start, int rc, uint32_t *bases,
                       uint32_t *nbits, uint32_t *sbits, int *bad);
__global__ void k_index_keys(SeqSetView T, int64_t nslots, int32_t step, SeedDesc sd, uint32_t sentinel,
                             uint32_t *keys, uint32_t *pos);
__global__ void k_offsets(const uint32_t *keys, int64_t n, uint32_t K, uint32_t *offsets);
__global__ void k_seed_count(const UnitDesc *units, const Chunk *chunks, SeqSetView Qp, SeqSetView Qm,
                             const uint32_t *offsets, SeedDesc sd, uint64_t *counts);
__global__ void k_seed_emit(const UnitDesc *units, const Chunk *chunks, SeqSetView Qp, SeqSetView Qm,
                            const uint32_t *offsets, const uint32_t *tpos, SeedDesc sd, const uint64_t *hit_off,
                            sfe_hit *out);
// ungapped X-drop of given hits, and the fused seed + X-drop over query chunks
void launch_xdrop_raw(const sfe_hit *hits, int64_t n, const QueryDesc *qd, int32_t nq, SeqSetView T, int64_t tb,
                      int64_t nt, SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc, int span, sfe_hsp *out, int *err,
                      hipStream_t st);
void launch_seed_xdrop(const UnitDesc *units, const Chunk *chunks, int64_t nch, SeqSetView T, int64_t tb, int64_t nt,
                       SeqSetView Qp, SeqSetView Qm, const uint32_t *offsets, const uint32_t *tpos, const SeedDesc &sd,
                       const ScoreDesc &sc, sfe_hsp *out, uint64_t cap, unsigned long long *counters, hipStream_t st);
__global__ void k_hsp_key(const sfe_hsp *h, const uint32_t *perm, int64_t n, int field, uint32_t *key);
__global__ void k_iota(uint32_t *a, int64_t n);

// k_sort.hip: stable LSD radix sort of (key, u32 value) pairs over key bits [0, end_bit), and the
// exclusive prefix sum; both count in 64 bits.  radix_temp_bytes / scan_work_words size their scratch.
template <typename K>
void radix_sort_pairs(const K *kin, K *kout, const uint32_t *vin, uint32_t *vout, int64_t n, int end_bit, void *temp,
                      hipStream_t st);
int64_t radix_temp_bytes(int64_t n, int key_bytes);
template <typename T, typename O>
void scan_exclusive(const T *in, O *out, int64_t n, uint64_t *work, hipStream_t st);
int64_t scan_work_words(int64_t n);
__global__ void k_hsp_unique_flags(const sfe_hsp *h, const uint32_t *perm, int64_t n, uint32_t *flag);
__global__ void k_hsp_compact(const sfe_hsp *h, const uint32_t *perm, const uint32_t *flag, const uint32_t *dst,
                              int64_t n, sfe_hsp *out);

__global__ void k_nsum(const uint32_t *nbits, int64_t nwords, uint32_t *nsum);

// gapped stage (k_extend.hip)
void launch_make_tasks(const ExtItem *items, int64_t n, const UnitDesc *units, int64_t nt, HalfTask *tasks,
                       hipStream_t st, const int64_t *n_dev = nullptr);
void launch_sched_reset(uint32_t *bits, int32_t nwords, int32_t *avail, int32_t avail0, unsigned int *qhead,
                        unsigned long long *run_head, hipStream_t st);
// fused extension + traceback (k_fused.hip); plain: grid = wq.n blocks, one
// half each; persistent: `grid` waves pulling halves from the queue
// kcap > 0: a half still running at antidiagonal kcap stops with HALF_LONG
// narrow: the packed 16-bit kernel (perm scores, Y-drop range checked by the
// caller; cells_per_lane rounds up to an even count)
// dyn_lds: dynamic LDS requested per block and left unused -- it caps how many
// blocks (waves) a compute unit takes, so a persistent grid spreads evenly
void launch_ydrop_fused(int cells_per_lane, bool perm, bool narrow, bool persistent, const HalfTask *tasks,
                        WorkQueue wq, int64_t grid, SeqSetView T, SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc,
                        ChunkPool pool, RunArena ra, HalfResult *res, int kcap, size_t dyn_lds, hipStream_t st);
// A group of 4 waves per half (wave-group window of 256 * cells_per_lane rows,
// cells_per_lane 2 or 4), one block per half ids[0 .. n).
void launch_ydrop_coop(int cells_per_lane, bool perm, const HalfTask *tasks, const int32_t *ids, int64_t n,
                       SeqSetView T, SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc, ChunkPool pool, RunArena ra,
                       HalfResult *res, hipStream_t st);
int ydrop_fused_blocks_per_cu(int cells_per_lane, bool perm, bool narrow, bool persistent, size_t dyn_lds);
void launch_ydrop_ring(const HalfTask *tasks, const int32_t *ids, int64_t n, SeqSetView T, SeqSetView Qp,
                       SeqSetView Qm, const ScoreDesc &sc, Arena arena, int32_t *ring, int32_t cap_rows,
                       HalfResult *res, hipStream_t st);
void launch_assemble(const ExtItem *items, int64_t n, const UnitDesc *units, const HalfResult *res,
                     SeqSetView T, SeqSetView Qp, SeqSetView Qm, const ScoreDesc &sc, sfe_aln *out,
                     hipStream_t st);
void launch_traceback(const HalfResult *res, const int32_t *half_ids, int64_t n, Arena arena,
                      const uint64_t *run_off, uint32_t *runs, uint32_t *nruns, hipStream_t st);
void launch_ops_assemble(const int32_t *item_ids, int64_t n, const uint64_t *run_off, const uint32_t *runs,
                         const uint32_t *nruns, const uint64_t *ops_off, uint32_t *ops, uint32_t *nops,
                         hipStream_t st);

// learned cost model (k_learn.hip)
void launch_mlp_round(const float *master, uint16_t *p16, hipStream_t st);
void launch_mlp_forward(const float *X, int64_t n, const uint16_t *p16, float *Y, hipStream_t st);
void launch_mlp_grad(const float *X, const float *T, const int32_t *ids, int32_t B, const uint16_t *p16,
                     float *part, float *sse, hipStream_t st);
void launch_mlp_apply(const float *part, int nb, const float *sse, int32_t B, float *grad, float *master, float *m,
                      float *v, uint16_t *p16, float lr, float c1, float c2, float *loss, hipStream_t st);
void launch_hsp_features(const sfe_hsp *h, int64_t n, const int32_t *unit_of, const UnitDesc *units, SeqSetView T,
                         int64_t nt, SeqSetView Qp, SeqSetView Qm, const uint32_t *order, const uint32_t *okey,
                         const int64_t *ustart, const int64_t *uend, float *F, hipStream_t st);
void launch_hsp_anchor_keys(const sfe_hsp *h, int64_t n, const int32_t *unit_of, uint64_t *key, uint32_t *ids,
                            hipStream_t st);
void launch_hsp_unit_ranges(const sfe_hsp *h, const int32_t *unit_of, const uint32_t *order, int64_t n,
                            uint32_t *okey, int64_t *ustart, int64_t *uend, hipStream_t st);

}  // namespace sfe
