/*
 * sfe.h -- C ABI of the MI355X (gfx950) seed -> filter -> extend library.
 *
 * The library computes the data-parallel core of the seed-filter-extend
 * pipeline of Sundram, "Dependencies and Dataflow in Seed-Filter-Extend
 * Pipelines" (2026): spaced-seed hits of query windows against a target
 * position table (Sec. 1, Sec. 7), the ungapped X-drop filter on every hit
 * (Sec. 3, Sec. 8), and gapped Y-drop extension of the surviving candidate
 * regions, each anchor extended as two halves (Sec. 8), committed with the
 * semantics of the strict serial algorithm (Alg. 1) while the extensions run
 * speculatively in batches (Alg. 3, Sec. 5).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Sequences are ASCII: A C G T (upper case), a c g t (soft-masked), N/n and
 *   the IUPAC ambiguity letters R Y S W K M B D H V (scored as N).  Any other
 *   byte is SFE_EINVAL.  Residue pointers may be host or device memory.
 * - Coordinates are 0-based, half-open, uint32.  Strand 0 is the query as
 *   given; strand 1 is its reverse complement and its coordinates are taken
 *   in reverse-complement space (position p of the minus strand is base
 *   length-1-p of the query, complemented).
 * - Output buffers may be host or device memory; the library copies into
 *   them with unified addressing.  Calls are ordered on the context's stream
 *   and return only when their results are in the caller's buffers.
 * - Capacity protocol: when an output capacity is too small, nothing is
 *   written, *n_out receives the required count, and SFE_ECAPACITY returns.
 * - Ownership: contexts and indexes belong to the library until destroyed;
 *   inputs are borrowed for the duration of the call; outputs belong to the
 *   caller.
 * - Scores are int32.  A call in which any ungapped or gapped score reaches
 *   2^29 stops with SFE_ERANGE (this keeps every intermediate value inside
 *   int32); so does a sequence longer than 2^32 - 64 bases.
 * - No call throws; on failure the status is returned and sfe_last_error()
 *   describes it.
 */
#ifndef SFE_H
#define SFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sfe_status;
#define SFE_OK 0
#define SFE_EINVAL (-1)     /* malformed argument (pattern, letter, scoring, null pointer) */
#define SFE_ENOMEM (-2)     /* device or host allocation failed */
#define SFE_ECAPACITY (-3)  /* an output buffer is too small; *n_out holds the need */
#define SFE_ERANGE (-4)     /* a sequence breaks the int32 score or uint32 coordinate range */
#define SFE_EDEVICE (-5)    /* a HIP runtime call failed */
#define SFE_EINTERNAL (-6)  /* an internal consistency check failed */
#define SFE_EIO (-7)        /* a file could not be opened, read or written */

typedef struct sfe_ctx sfe_ctx;
typedef struct sfe_index sfe_index;

/* A spaced seed (Sec. 7): pattern of '1' (care) and '0' (don't care), first
 * and last characters '1', span <= 32, weight (number of '1') <= 14.  The
 * weight cap comes from the position table's dense offsets array, 4^weight + 1
 * u32 entries: 1 GiB at weight 14, 16 GiB at 16 -- the paper's seeds (weight
 * 12 of span 19, and 14 of 22) fit. 
 * transitions = 1 also accepts windows whose care positions differ in exactly
 * one place by a transition (A<->G, C<->T).  A target position p is indexed
 * iff p % step == 0. */
typedef struct {
    const char *pattern;
    int32_t transitions;
    int32_t step;
} sfe_seed_spec;

/* Integer scoring: sub[a][b] for target base a and query base b in the order
 * A C G T N; a gap of length L costs gap_open + L * gap_extend.  |sub| < 2^15,
 * 0 <= gap_open < 2^20, 0 < gap_extend < 2^15, 0 <= xdrop, ydrop < 2^29. */
typedef struct {
    int32_t sub[5][5];
    int32_t gap_open, gap_extend;
    int32_t xdrop;          /* ungapped extension stops once best - running > xdrop */
    int32_t hsp_thresh;     /* an HSP passes the filter when its score >= hsp_thresh */
    int32_t ydrop;          /* a DP cell is pruned when H < (best so far) - ydrop */
    int32_t gapped_thresh;  /* an extension is committed when its score >= gapped_thresh */
} sfe_scoring;

typedef struct {
    const char *residues;   /* host or device pointer to `length` ASCII bytes */
    int64_t length;
} sfe_seq;

/* One seed hit: target window start t, query window start q (strand space). */
typedef struct {
    uint32_t t, q, query_id;
    uint8_t strand, pad[3];
} sfe_hit;                  /* 16 bytes */

/* One ungapped segment: target [t0, t0+len), query [q0, q0+len). */
typedef struct {
    uint32_t t0, q0, len;
    int32_t score;
    uint32_t query_id;
    uint8_t strand, pad[3];
} sfe_hsp;                  /* 24 bytes */

/* One gapped alignment.  ops[ops_offset .. ops_offset+ops_len) are
 * run-length edit operations (len << 2 | op), op 0 = M (a column consuming
 * one target and one query base), 1 = I (consumes query only), 2 = D
 * (consumes target only), read from (t_start, q_start) to (t_end, q_end).
 * cells = DP cells computed by the two halves; flags bit 0 = score reached
 * gapped_thresh. */
typedef struct {
    uint32_t t_start, t_end, q_start, q_end;
    int32_t score;
    uint32_t query_id;
    uint32_t anchor_t, anchor_q;
    uint64_t ops_offset;
    uint64_t cells;
    uint32_t ops_len;
    uint8_t strand, flags, pad[2];
} sfe_aln;                  /* 56 bytes */

#define SFE_ALN_PASSED 1u

/* Schedules of the gapped extension; all give identical results. */
#define SFE_SCHED_PLAIN 0       /* one wavefront per anchor-half, one launch per batch */
#define SFE_SCHED_PERSISTENT 1  /* persistent work-stealing launch over a cost-ordered queue */
#define SFE_SCHED_ADAPTIVE 2    /* plain launch for a batch of at least sfe_tuning.adaptive_halves
                                   halves, persistent below (fewer halves in flight at once,
                                   spread evenly over the SIMDs) */
#define SFE_SCHED_BINNED 3      /* learned binning with plain launches: one wavefront per half, the
                                   halves a cost model predicts to be long launched first (see
                                   sfe_align_opts.model), the rest in batch order */

/* Speculation policies of sfe_align; all give identical results.
 * PREFIX: each batch is the next round_k HSPs of a (query, strand) whose
 *   anchors are not contained in a committed alignment (Alg. 3 as printed).
 * DEFER:  the scan also passes over (defers) an HSP whose anchor lies on an M
 *   column of an earlier extension still waiting for commit, or whose
 *   diagonal is within near_band (32 by default) of an earlier HSP already in
 *   the batch while no extension computed so far spans the anchor's region
 *   (its bounding box); deferred HSPs are decided in later batches.  A waiting
 *   extension holds nothing back when it is expected to be skipped at commit:
 *   its anchor already lies in a committed alignment, or on an M column of an
 *   earlier waiting extension that is not itself expected to be skipped.
 *   Commit still walks the HSPs in order and stops at the first one without
 *   an extension. */
#define SFE_POLICY_DEFER 0
#define SFE_POLICY_PREFIX 1

typedef struct {
    int32_t round_k;        /* per (query, strand) extensions per batch; <= 0 picks a default */
    int32_t schedule;       /* SFE_SCHED_* */
    int32_t strands;        /* bit 0 plus, bit 1 minus; 0 means both */
    int32_t max_cells_per_lane; /* 0 = automatic (6); 2, 3, 4, 6 or 8 rows per lane (64 x that many rows)
                               in the first band window; wider bands move on to 8, then to the
                               workgroup kernel */
    int32_t policy;         /* SFE_POLICY_* */
    int32_t near_band;      /* SFE_POLICY_DEFER's nearness rule: diagonals within which a later HSP
                               of the batch waits for an earlier one; 0 = 32, < 0 = rule off
                               (round_k 0 then means 256: without the rule the first batch would
                               hold every HSP of every region at once) */
    int64_t arena_bytes;    /* device memory for traceback codes of the halves in flight,
                               allocated once per context; 0 = half the free device memory
                               at first use (at least 32 GiB).  A batch whose halves
                               need more at once runs with fewer in flight; a single half
                               that needs more makes the arena grow. */
    const struct sfe_model *model; /* NULL, or a cost model: with SFE_SCHED_PERSISTENT,
                               SFE_SCHED_ADAPTIVE or SFE_SCHED_BINNED the halves of each batch
                               predicted to compute at least 2^20 cells are queued (or launched)
                               first, longest first, the rest in batch order.  Never changes the
                               output. */
    int32_t filter;         /* SFE_FILTER_XDROP (0, default) or SFE_FILTER_YDROP */
    int32_t pad;
} sfe_align_opts;

/* Filters of sfe_align.  XDROP: the ungapped X-drop extension of every seed
 * hit (Sec. 3, Sec. 8).  YDROP: the two-dimensional filter the paper proposes
 * in its place (Sec. 8, Sec. 9): both gapped halves of every hit around the
 * middle column of its seed window, pruned with Y := xdrop (sfe_gapped_ydrop's
 * rules); a hit whose total reaches hsp_thresh becomes an HSP spanning its
 * seed window (t, q, span) with that total as score, and the pipeline goes on
 * as with X-drop HSPs.  sfe_stats.xdrop_columns then counts the filter's DP
 * cells. */
#define SFE_FILTER_XDROP 0
#define SFE_FILTER_YDROP 1

/* The options sfe_align runs with: *in (NULL: all zero) with every automatic
 * field filled in -- strands 3; max_cells_per_lane 6 (others clamped into
 * [2, 8]); near_band 32 (negative: -1, rule off); round_k 2^20 under
 * SFE_POLICY_DEFER with the nearness rule on, otherwise 256 (Alg. 3's batch
 * size; the paper settles on 48 to 64 for CPU threads).  SFE_EINVAL for an
 * unknown schedule or policy or a negative field that has no meaning.  Host
 * only: touches no device, so it also checks options before a context exists. */
sfe_status sfe_align_opts_resolve(const sfe_align_opts *in, sfe_align_opts *out);

typedef struct {
    int64_t seed_hits;          /* hits evaluated by the X-drop filter */
    int64_t hsps_raw;           /* hits whose X-drop score passed */
    int64_t hsps;               /* unique passing HSPs */
    int64_t rounds;             /* speculative batches (Alg. 3 rounds) */
    int64_t extensions;         /* gapped extensions computed (both halves = one) */
    int64_t committed;          /* alignments committed */
    int64_t shadow;             /* extensions discarded at commit because their anchor was contained */
    int64_t cells;              /* DP cells of all computed extensions */
    int64_t overflow_reruns;    /* halves re-run with a wider band or a larger arena */
    int64_t xdrop_columns;      /* columns scored by the X-drop filter (seed span included) */
    int64_t ydrop_launches;     /* launches of the gapped-extension kernel */
    int64_t ydrop_kernel_cells; /* DP cells computed by those launches */
    int64_t seed_xdrop_launches;/* launches of the fused seed + X-drop kernel */
    double ms_seed_xdrop, ms_hsp_set, ms_extend, ms_total;   /* host wall clock per stage */
    double ms_ydrop_kernel;     /* sum of HIP-event durations of the gapped-extension launches */
    double ms_seed_xdrop_kernel;/* sum of HIP-event durations of the fused seed + X-drop launches */
    int64_t predicted_halves;   /* halves queued by a cost model */
    int64_t mispredicted_halves;/* of those: predicted log2(1 + cells) off by more than 2 */
    double ms_predict;          /* host wall clock of features + model inference */
    int64_t narrow_launches;    /* of ydrop_launches: launches of the packed 16-bit kernel */
    int64_t graph_launches;     /* of ydrop_launches: first launches of a batch run as a replay of a
                                   recorded graph (tuning.use_graphs) */
    int64_t graph_records;      /* graphs recorded for them (the rest were replays of an earlier one) */
} sfe_stats;

/* Context on `device` using `hip_stream` (a hipStream_t, or NULL for a
 * stream of its own). */
sfe_status sfe_ctx_create(int device, void *hip_stream, sfe_ctx **out);
void sfe_ctx_destroy(sfe_ctx *ctx);

/* Position table of the target (Sec. 5 phase 1, Sec. 7): the 2-bit packed
 * target with N and soft-mask bit planes, and the list of indexed window
 * starts grouped by seed key (valid windows only: no N or soft-masked base in
 * the span), resident in device memory. */
sfe_status sfe_build_index(sfe_ctx *ctx, const sfe_seq *target, const sfe_seed_spec *seed,
                           sfe_index **out);
void sfe_index_destroy(sfe_index *idx);

/* All seed hits of the queries (Sec. 1, Sec. 7): (t, q) such that both
 * windows are valid and the care positions match exactly or, with
 * transitions, differ by one transition.  strands: bit 0 plus, bit 1 minus.
 * Output in (query_id, strand, q, t) order; each hit once. */
sfe_status sfe_seed_hits(sfe_ctx *ctx, const sfe_index *idx, const sfe_seq *queries, int32_t nq,
                         int32_t strands, sfe_hit *out, int64_t cap, int64_t *n_hits);

/* Ungapped X-drop extension of hits (Sec. 3, Sec. 8).  From the seed window
 * the scan runs right of it and left of it along the diagonal, stopping once
 * best - running > xdrop or at a sequence end; on ties the shorter extent is
 * kept.  With flags = SFE_XDROP_RAW, out[x] is the segment of hits[x] whatever
 * its score (exactly n records).  With flags = 0, out holds the passing
 * segments (score >= hsp_thresh) with exact duplicates removed, in the order
 * the serial algorithm walks them: query_id, score descending, strand, t0,
 * q0, len ascending. */
#define SFE_XDROP_RAW 1
sfe_status sfe_ungapped_xdrop(sfe_ctx *ctx, const sfe_index *idx, const sfe_seq *queries, int32_t nq,
                              const sfe_hit *hits, int64_t n, const sfe_scoring *sc, int32_t flags,
                              sfe_hsp *out, int64_t cap, int64_t *n_hsps);

/* Gapped Y-drop extension of each HSP (Sec. 8), without commit.  The anchor
 * is the HSP's middle column (offset (len-1)/2), part of the alignment; the
 * forward half extends from the next column on, the backward half from the
 * previous column backwards.  Each half is an affine-gap DP over
 * antidiagonals; a cell is live when H >= (best over earlier antidiagonals)
 * - ydrop; the half stops after two antidiagonals with no live cell; its end
 * is the first live cell (smallest antidiagonal, then smallest target offset)
 * reaching its best.  out[x] is the alignment of hsps[x] (exactly n records);
 * edit operations are written only for records with SFE_ALN_PASSED. */
sfe_status sfe_gapped_ydrop(sfe_ctx *ctx, const sfe_index *idx, const sfe_seq *queries, int32_t nq,
                            const sfe_hsp *hsps, int64_t n, const sfe_scoring *sc,
                            sfe_aln *out, uint32_t *ops, int64_t ops_cap, int64_t *n_ops);

/* The whole pipeline with the commit semantics of Alg. 1 (Sec. 4), run as
 * Alg. 3 (Sec. 5): per (query, strand), HSPs are walked in the order of
 * sfe_ungapped_xdrop; an HSP whose anchor column lies on an M column of an
 * alignment already committed is skipped; batches of up to round_k unskipped
 * HSPs are extended speculatively and committed in order, re-checking the
 * anchor against every earlier commit.  The result does not depend on
 * round_k or on the schedule.  Output order: query_id, strand, t_start,
 * q_start, t_end, q_end, anchor_t, anchor_q.  stats may be NULL. */
sfe_status sfe_align(sfe_ctx *ctx, const sfe_index *idx, const sfe_seq *queries, int32_t nq,
                     const sfe_scoring *sc, const sfe_align_opts *opts,
                     sfe_aln *out, int64_t cap, int64_t *n_alns,
                     uint32_t *ops, int64_t ops_cap, int64_t *n_ops, sfe_stats *stats);

/* Schedule knobs of a context (an autotuner's output; none changes results).
 * wave_group_cap: a half still running after this many antidiagonals on one
 *   wavefront restarts on a group of 4 wavefronts that share its band (one LDS
 *   barrier per antidiagonal, Sec. 8's cooperative mapping); halves a cost
 *   model predicts to be longer start there.  0 = never (default). */
typedef struct {
    int32_t wave_group_cap;
    int32_t use_graphs;     /* 1: sfe_model_train records its whole step sequence in one hipGraph
                               and launches it once; sfe_align runs the first one-wave launch of
                               every batch (pool and queue reset, half tasks, fused extension) as
                               a recorded graph that reads the item and half counts from device
                               memory, replayed while buffers, scores and launch shape stay the
                               same (buffers then sized for the next power of two of the batch;
                               a plain launch covers that capacity and its extra waves exit at
                               once).  Same kernels, same results; if recording fails, stream
                               launches from then on. */
    int32_t wide_scores;    /* 1: gapped extension always in 32-bit arithmetic; 0 (default): in
                               packed 16-bit arithmetic, values relative to the Y-drop threshold,
                               when every score fits in int8 and ydrop + gap_open + gap_extend +
                               2 * max |score| + 512 <= 32767 (same results either way) */
    int32_t persist_waves_per_cu; /* waves per compute unit of a persistent launch (capped by
                               occupancy); 0 = 8, two per SIMD */
    int32_t adaptive_halves;  /* SFE_SCHED_ADAPTIVE threshold in halves; 0 = 131072 */
    int32_t reserved[3];
} sfe_tuning;
sfe_status sfe_ctx_set_tuning(sfe_ctx *ctx, const sfe_tuning *t);
sfe_status sfe_ctx_get_tuning(const sfe_ctx *ctx, sfe_tuning *t);

/* Autotuner.  Times sfe_align on a sample of the workload (the first
 * sample_bases of every query, all against idx) under each candidate schedule
 * -- rows per lane 4 / 6 in the first band window; plain, persistent,
 * adaptive or binned launch, only the last three (with the model) when
 * opts->model is given; 8 or 16 waves per compute unit for the persistent
 * grid; wave groups
 * for long halves off or after 8192 antidiagonals -- three times each, and
 * keeps the fastest (by its best time): the context's wave_group_cap and
 * persist_waves_per_cu are set and opts->max_cells_per_lane / schedule are
 * written.  Other fields of *opts are used as given.  report (may be NULL)
 * receives every candidate's extension time.  No choice changes results. */
typedef struct {
    int32_t cells_per_lane, schedule, wave_group_cap, waves_per_cu;
    double ms_extend;
} sfe_tune_entry;
typedef struct {
    int32_t n, best;
    sfe_tune_entry entries[32];
} sfe_tune_report;
sfe_status sfe_autotune(sfe_ctx *ctx, const sfe_index *idx, const sfe_seq *queries, int32_t nq,
                        const sfe_scoring *sc, int64_t sample_bases, sfe_align_opts *opts,
                        sfe_tune_report *report);

/* ---------------------------------------------------------------------------
 * Learned cost model.  The cost of an anchor-half is unknown until it has run
 * (Sec. 8) and sorting work by expected size up front is the load-balancing
 * step Sec. 9 leaves open; this library predicts it with a small MLP of its
 * own design.  Parameters (SFE_MLP_NPARAMS floats, FP32 master copy), in this
 * order, row-major out x in: W1 64x16, b1 64, W2 64x64, b2 64, W3 64x64, b3 64,
 * W4 4x64, b4 4.  Forward: parameters and inputs rounded to BF16 (nearest even),
 * A = bf16(relu(X W^T + b)) per hidden layer with FP32 accumulation, linear
 * FP32 output.  Loss: mean of (Y - T)^2 over the batch and the 4 outputs;
 * back-propagated signals are rounded to BF16 before each product, gradients
 * accumulate in FP32; Adam (0.9, 0.999, 1e-8) on the master weights.
 * Outputs / targets per HSP: log2(1 + cells) and log2(1 + i* + j*) of the
 * forward half, then the same of the backward half.
 *
 * Features (SFE_MLP_NFEAT floats per HSP; neighbours are the other HSPs of
 * the same call with the same query and strand; anchors per the HSP anchor
 * rule of sfe_gapped_ydrop; windows clip at sequence ends):
 *   0 score/4096          1 log2(1+len)/16       2 identical columns/len
 *   3 transition columns/len  4 other mismatch or N columns/len
 *   5 (t0-q0)/target length   6 strand            7 anchor t/target length
 *   8 anchor q/query length   9, 10 GC fraction of the non-N bases within
 *   1000 of the anchor (target, query)  11 log2(1+#neighbours with |dt| <= 5000
 *   and |d diagonal| <= 64)/8  12 log2(1+#neighbours with |dt| <= 10000)/8
 *   13 log2(1+smallest dt in (0, 10000] with |d diagonal| <= 64)/16, else 1
 *   14 the same upstream (dt < 0)   15 soft-masked fraction of the target
 *   within 1000 of the anchor  (dt = anchor t difference). */
#define SFE_MLP_NFEAT 16
#define SFE_MLP_NOUT 4
#define SFE_MLP_NPARAMS 9668
typedef struct sfe_model sfe_model;

/* features: n x SFE_MLP_NFEAT (host or device). */
sfe_status sfe_hsp_features(sfe_ctx *ctx, const sfe_index *idx, const sfe_seq *queries, int32_t nq,
                            const sfe_hsp *hsps, int64_t n, float *features);
/* Training log of the plain pipeline: the features of each HSP and the
 * targets (n x SFE_MLP_NOUT) of its gapped extension. */
sfe_status sfe_extension_log(sfe_ctx *ctx, const sfe_index *idx, const sfe_seq *queries, int32_t nq,
                             const sfe_hsp *hsps, int64_t n, const sfe_scoring *sc,
                             float *features, float *targets);
/* A model on ctx's device with the given initial parameters (host or device).
 * It runs on ctx's stream: destroy it before ctx (destroying it after ctx is
 * allowed; using it is not). */
sfe_status sfe_model_create(sfe_ctx *ctx, const float *params, sfe_model **out);
void sfe_model_destroy(sfe_model *m);
sfe_status sfe_model_params(const sfe_model *m, float *params);
/* y (n x SFE_MLP_NOUT) from x (n x SFE_MLP_NFEAT). */
sfe_status sfe_model_predict(sfe_model *m, const float *x, int64_t n, float *y);
/* Gradient (SFE_MLP_NPARAMS) and loss of the whole set (x, t) as one batch. */
sfe_status sfe_model_grad(sfe_model *m, const float *x, const float *t, int64_t n, float *grad, float *loss);
/* sfe_model_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same results, but no allocation of any kind.  x
 * (n x SFE_MLP_NFEAT), t (n x SFE_MLP_NOUT), grad (SFE_MLP_NPARAMS) and loss
 * (1 float) must be device memory; 1 <= n <= SFE_NOALLOC_MAX_SAMPLES
 * (SFE_EINVAL otherwise).  The working memory (sample ids, per-block partial
 * gradients: about 10 MB) is one fixed array per device, set up when a
 * context is created on that device and shared by every call there: calls
 * that overlap on one device race.  The call is ordered on the context's
 * stream and returns without waiting for it. */
#define SFE_NOALLOC_MAX_SAMPLES 16384
sfe_status sfe_model_grad_noalloc(sfe_model *m, const float *x, const float *t, int64_t n, float *grad,
                                  float *loss);
/* Adam steps over the batches of `order` (n_order sample ids in [0, n),
 * consumed `batch` at a time, a short last batch used as is); losses (one per
 * step, may be NULL) receives each batch's loss before its update. */
sfe_status sfe_model_train(sfe_model *m, const float *x, const float *t, int64_t n, const int32_t *order,
                           int64_t n_order, int32_t batch, float lr, float *losses);
/* Persistence (a versioned blob): a 32-byte header -- magic "SFEMLP\0\0",
 * u32 version 1, u32 layout 1 (the 16-64-64-64-4 network above), u32
 * parameter count SFE_MLP_NPARAMS, u32 0, i64 Adam steps taken -- then the
 * FP32 master parameters, the Adam first and second moments (SFE_MLP_NPARAMS
 * floats each) and a u64 FNV-1a hash of all preceding bytes; little-endian,
 * 116056 bytes.  A loaded model continues training exactly where the saved
 * one stopped.  sfe_model_load with ctx and out both NULL only checks the
 * file.  Errors: SFE_EIO (cannot open, read or write), SFE_EINVAL (not a model
 * file of this version and layout: wrong size, magic, header or hash). */
sfe_status sfe_model_save(const sfe_model *m, const char *path);
sfe_status sfe_model_load(sfe_ctx *ctx, const char *path, sfe_model **out);

const char *sfe_status_str(sfe_status s);
const char *sfe_last_error(const sfe_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* SFE_H */
