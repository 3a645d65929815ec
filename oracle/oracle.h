/*
 * oracle.h -- interface of the CPU oracle (test infrastructure only; the HIP
 * library never includes this file and this file includes nothing of it).
 * Sequences are arrays of codes 0..3 = A,C,G,T and 4 = N, with a parallel
 * array of soft-mask flags.  All coordinates are 0-based.
 */
#ifndef SFE_ORACLE_H
#define SFE_ORACLE_H
#include <stdint.h>

typedef struct {
    int32_t sub[5][5];          /* substitution scores, rows/cols A C G T N */
    int32_t gap_open, gap_extend;
    int32_t xdrop, hsp_thresh, ydrop, gapped_thresh;
} orc_scoring;

typedef struct { int64_t t0, q0, len; int64_t score; int64_t work; } orc_hsp;

typedef struct { int32_t best; int32_t pad; int64_t i_end, j_end, cells, n_ops; } orc_half;

typedef struct {
    int64_t t_start, t_end, q_start, q_end;
    int64_t score;
    int64_t anchor_t, anchor_q;
    int64_t cells;
    int64_t ops_off, ops_len;
    int32_t query_id, strand;
} orc_aln;

typedef struct {
    orc_aln *alns; int64_t n_alns, cap_alns;
    uint32_t *ops; int64_t n_ops, cap_ops;
    int64_t n_extensions;       /* gapped extensions computed */
    int64_t ext_cells;          /* DP cells of those extensions */
} orc_result;

int orc_encode(const char *txt, int64_t n, uint8_t *code, uint8_t *soft);
void orc_revcomp(const uint8_t *code, const uint8_t *soft, int64_t n, uint8_t *rcode, uint8_t *rsoft);
int64_t orc_seed_hits(const uint8_t *tc, const uint8_t *ts, int64_t nt,
                      const uint8_t *qc, const uint8_t *qs, int64_t nq,
                      const char *pattern, int32_t transitions, int32_t step,
                      uint32_t *out_t, uint32_t *out_q, int64_t cap);
void orc_xdrop(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
               int64_t t, int64_t q, int32_t span, const orc_scoring *sc, orc_hsp *out);
void orc_xdrop_batch(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
                     const uint32_t *t, const uint32_t *q, int64_t n, int32_t span,
                     const orc_scoring *sc, orc_hsp *out);
int64_t orc_ydrop_half(const uint8_t *A, int64_t nA, const uint8_t *B, int64_t nB,
                       const orc_scoring *sc, orc_half *res, uint8_t *ops, int64_t ops_cap);
int64_t orc_extend(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
                   int64_t ta, int64_t qa, const orc_scoring *sc, orc_aln *out,
                   uint32_t *ops, int64_t ops_cap);
void orc_commit_unit(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
                     const orc_hsp *hsps, int64_t n, const orc_scoring *sc,
                     int64_t K, int32_t query_id, int32_t strand, orc_result *res);
orc_result *orc_result_new(void);
void orc_result_free(orc_result *r);

#endif
