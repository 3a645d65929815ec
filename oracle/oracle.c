/*
 * oracle.c -- plain, slow, single-threaded CPU oracle for the seed -> filter
 * (ungapped X-drop) -> extend (gapped Y-drop) pipeline of "Dependencies and
 * Dataflow in Seed-Filter-Extend Pipelines" (Sundram, 2026).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library: every definition below is written out again from the paper, and
 * where the paper is silent from a stated reading of it (given beside the
 * code that uses it).
 *
 * Every integer in the dynamic programs is int32 semantics with the sentinel
 * NEG = -2^30; intermediate sums are formed in int64 and clamped at NEG so
 * that nothing here can overflow.
 *
 * Sections (paper):
 *   Sec. 1  seeds over a position table, local DP at candidate regions
 *   Sec. 4  Alg. 1 (the strict serial walk): an HSP whose anchor is covered
 *           by an earlier commit is passed over, others are extended and
 *           committed when they reach the gapped threshold
 *   Sec. 5  Alg. 3 (speculative): batches of up to K uncovered HSPs are
 *           extended independently and committed in order, the anchor test
 *           re-applied at commit
 *   Sec. 7  the 12-of-19 spaced seed 1110100110010101111, transition tolerance
 *   Sec. 8  X-drop is a 1-D DP without gaps; Y-drop stops when the score
 *           falls a fixed amount below the best; anchors are extended as two
 *           halves.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define NEG (-(1 << 30))

static int32_t clampneg(int64_t v) { return v < NEG ? NEG : (int32_t)v; }
static int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

/* ------------------------------------------------------------------------ */
/* Alphabet: A0 C1 G2 T3, N (and IUPAC ambiguity letters) 4;                */
/* lower case marks a soft-masked base.                                      */
/* ------------------------------------------------------------------------ */
int orc_encode(const char *txt, int64_t n, uint8_t *code, uint8_t *soft)
{
    for (int64_t p = 0; p < n; p++) {
        char c = txt[p];
        int lower = (c >= 'a' && c <= 'z');
        char u = lower ? (char)(c - 'a' + 'A') : c;
        int v;
        switch (u) {
        case 'A': v = 0; break;
        case 'C': v = 1; break;
        case 'G': v = 2; break;
        case 'T': v = 3; break;
        case 'N': case 'R': case 'Y': case 'S': case 'W': case 'K':
        case 'M': case 'B': case 'D': case 'H': case 'V':
            v = 4; break;
        default:
            return -1;
        }
        code[p] = (uint8_t)v;
        soft[p] = (uint8_t)lower;
    }
    return 0;
}

/* Minus strand: reverse complement, A<->T, C<->G, N stays N; coordinates  */
/* are taken in reverse-complement space; soft-mask flags move with bases.  */
void orc_revcomp(const uint8_t *code, const uint8_t *soft, int64_t n,
                 uint8_t *rcode, uint8_t *rsoft)
{
    for (int64_t p = 0; p < n; p++) {
        uint8_t c = code[n - 1 - p];
        rcode[p] = (c == 4) ? 4 : (uint8_t)(3 - c);
        rsoft[p] = soft[n - 1 - p];
    }
}

/* ------------------------------------------------------------------------ */
/* Spaced seeds (Sec. 7).  A target position is indexed iff it is a multiple */
/* of the step (default 1).                                                   */
/* ------------------------------------------------------------------------ */
static int parse_pattern(const char *pat, int32_t *care, int32_t *span)
{
    int32_t s = 0, w = 0;
    for (; pat[s]; s++) {
        if (pat[s] == '1') {
            if (w >= 16) return -1;
            care[w++] = s;
        } else if (pat[s] != '0') {
            return -1;
        }
        if (s >= 32) return -1;
    }
    if (w == 0 || pat[0] != '1' || pat[s - 1] != '1') return -1;
    *span = s;
    return w;
}

/* a window is valid iff it fits and no base of its whole span (not only the
 * care positions) is N or soft-masked */
static int window_valid(const uint8_t *code, const uint8_t *soft, int64_t n, int64_t p, int32_t span)
{
    if (p < 0 || p + span > n) return 0;
    for (int32_t u = 0; u < span; u++)
        if (code[p + u] == 4 || soft[p + u]) return 0;
    return 1;
}

/* the codes at the care positions, first care position most significant */
static uint32_t window_key(const uint8_t *code, int64_t p, const int32_t *care, int32_t w)
{
    uint32_t key = 0;
    for (int32_t c = 0; c < w; c++) key = (key << 2) | code[p + care[c]];
    return key;
}

typedef struct { uint32_t key; uint32_t pos; } keypos;

static int cmp_keypos(const void *a, const void *b)
{
    const keypos *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
    return 0;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y);
}

/* The hits of one query strand against the target.  (t, q) is a hit iff both
 * windows are valid, t is a multiple of the step, and over the care positions
 * either every pair of bases is equal, or (transitions allowed) exactly one
 * pair differs and that pair is a transition (A<->G or C<->T: codes differ by
 * the bit 2).  The position table is a list of (key, t) sorted by a library
 * sort; lookups are binary searches.  Output order is (q, t) ascending.
 * Returns the number of hits (written up to cap), or -1 on a bad pattern. */
int64_t orc_seed_hits(const uint8_t *tc, const uint8_t *ts, int64_t nt,
                      const uint8_t *qc, const uint8_t *qs, int64_t nq,
                      const char *pattern, int32_t transitions, int32_t step,
                      uint32_t *out_t, uint32_t *out_q, int64_t cap)
{
    int32_t care[16], span;
    int32_t w = parse_pattern(pattern, care, &span);
    if (w < 0 || step < 1) return -1;

    int64_t nwin = nt >= span ? nt - span + 1 : 0;
    keypos *table = malloc(sizeof(keypos) * (size_t)(nwin > 0 ? nwin : 1));
    int64_t ntab = 0;
    for (int64_t p = 0; p < nwin; p++) {
        if (p % step != 0) continue;
        if (!window_valid(tc, ts, nt, p, span)) continue;
        table[ntab].key = window_key(tc, p, care, w);
        table[ntab].pos = (uint32_t)p;
        ntab++;
    }
    qsort(table, (size_t)ntab, sizeof(keypos), cmp_keypos);

    int64_t nhit = 0;
    uint32_t *buf = NULL;
    int64_t bufcap = 0;
    for (int64_t q = 0; q + span <= nq; q++) {
        if (!window_valid(qc, qs, nq, q, span)) continue;
        uint32_t key0 = window_key(qc, q, care, w);
        int64_t nb = 0;
        for (int32_t v = -1; v < (transitions ? w : 0); v++) {
            uint32_t key = key0;
            if (v >= 0) key ^= 2u << (2 * (w - 1 - v));   /* one transition at care position v */
            /* lower bound of key in table */
            int64_t lo = 0, hi = ntab;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (table[mid].key < key) lo = mid + 1; else hi = mid;
            }
            for (int64_t x = lo; x < ntab && table[x].key == key; x++) {
                if (nb == bufcap) {
                    bufcap = bufcap ? 2 * bufcap : 1024;
                    buf = realloc(buf, sizeof(uint32_t) * (size_t)bufcap);
                }
                buf[nb++] = table[x].pos;
            }
        }
        qsort(buf, (size_t)nb, sizeof(uint32_t), cmp_u32);
        for (int64_t x = 0; x < nb; x++) {
            if (nhit < cap) {
                out_t[nhit] = buf[x];
                out_q[nhit] = (uint32_t)q;
            }
            nhit++;
        }
    }
    free(buf);
    free(table);
    return nhit;
}

/* ------------------------------------------------------------------------ */
/* Ungapped X-drop filter (Sec. 3, Sec. 8: a 1-D DP without gaps).  Scans  */
/* stop once best - running > X (strict); the shortest best extent wins     */
/* ties (strict > update); scans stop at the sequence ends; an HSP passes   */
/* when its score is >= the HSP threshold.                                  */
/* ------------------------------------------------------------------------ */
static int32_t subst(const orc_scoring *sc, uint8_t a, uint8_t b) { return sc->sub[a][b]; }

void orc_xdrop(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
               int64_t t, int64_t q, int32_t span, const orc_scoring *sc, orc_hsp *out)
{
    int64_t work = span;
    int64_t s0 = 0;
    for (int32_t u = 0; u < span; u++) s0 += subst(sc, tc[t + u], qc[q + u]);

    /* right of the seed */
    int64_t s = 0, bR = 0, R = 0;
    for (int64_t r = 1; t + span - 1 + r < nt && q + span - 1 + r < nq; r++) {
        s += subst(sc, tc[t + span - 1 + r], qc[q + span - 1 + r]);
        work++;
        if (s > bR) { bR = s; R = r; }
        else if (bR - s > sc->xdrop) break;
    }
    /* left of the seed */
    int64_t bL = 0, L = 0;
    s = 0;
    for (int64_t r = 1; t - r >= 0 && q - r >= 0; r++) {
        s += subst(sc, tc[t - r], qc[q - r]);
        work++;
        if (s > bL) { bL = s; L = r; }
        else if (bL - s > sc->xdrop) break;
    }
    out->t0 = t - L;
    out->q0 = q - L;
    out->len = L + span + R;
    out->score = s0 + bL + bR;
    out->work = work;
}

/* every hit of one strand: out[x] is the X-drop HSP of hit (t[x], q[x]) */
void orc_xdrop_batch(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
                     const uint32_t *t, const uint32_t *q, int64_t n, int32_t span,
                     const orc_scoring *sc, orc_hsp *out)
{
    for (int64_t x = 0; x < n; x++) orc_xdrop(tc, nt, qc, nq, t[x], q[x], span, sc, &out[x]);
}

/* ------------------------------------------------------------------------ */
/* Gapped Y-drop extension of one anchor half (Sec. 8).  A gap of length L  */
/* costs open + L * extend.                                                 */
/*                                                                          */
/* The half is a DP over A (target side) and B (query side), both read away */
/* from the anchor: element i of A is A(i) = a_base[dir * i] etc.  Cells    */
/* are evaluated antidiagonal by antidiagonal (k = i + j).  A cell is live  */
/* when its H is at least (best over earlier antidiagonals) - Y; a read of  */
/* a cell that was not computed, or is not live, yields NEG for H, E and F. */
/* ------------------------------------------------------------------------ */
typedef struct { const uint8_t *base; int64_t dir; } seqview;
static uint8_t at(seqview v, int64_t i) { return v.base[v.dir * i]; }

typedef struct { int32_t H, E, F; uint8_t live; } dpcell;
typedef struct { int64_t lo, hi, off; int64_t minlive, maxlive; } adiag;  /* hi < lo: empty */

typedef struct {
    adiag *ad;        /* one per antidiagonal 0..kmax */
    int64_t nad;
    dpcell *cells;
    int64_t ncells, capcells;
} dpstore;

static const dpcell *getcell(const dpstore *st, int64_t k, int64_t i)
{
    if (k < 0 || k >= st->nad) return NULL;
    const adiag *a = &st->ad[k];
    if (a->hi < a->lo || i < a->lo || i > a->hi) return NULL;
    const dpcell *c = &st->cells[a->off + (i - a->lo)];
    return c->live ? c : NULL;
}
static int64_t getH(const dpstore *st, int64_t k, int64_t i) { const dpcell *c = getcell(st, k, i); return c ? c->H : NEG; }
static int64_t getE(const dpstore *st, int64_t k, int64_t i) { const dpcell *c = getcell(st, k, i); return c ? c->E : NEG; }
static int64_t getF(const dpstore *st, int64_t k, int64_t i) { const dpcell *c = getcell(st, k, i); return c ? c->F : NEG; }

static void emit(uint8_t **ops, int64_t *nops, int64_t *cap, uint8_t op)
{
    if (*nops == *cap) {
        *cap = *cap ? 2 * *cap : 256;
        *ops = realloc(*ops, (size_t)*cap);
    }
    (*ops)[(*nops)++] = op;
}

/* Runs one half.  On return *ops holds the traceback in emission order
 * (from the end cell back to the anchor), one byte per step: 0 M, 1 I, 2 D. */
static void ydrop_half(seqview A, int64_t nA, seqview B, int64_t nB, const orc_scoring *sc,
                       orc_half *res, uint8_t **ops, int64_t *nops, int64_t *opscap)
{
    const int64_t o = sc->gap_open, e = sc->gap_extend, oe = o + e, Y = sc->ydrop;
    dpstore st;
    int64_t kmax = nA + nB;
    st.ad = malloc(sizeof(adiag) * (size_t)(kmax + 1));
    st.nad = 0;
    st.capcells = 1024;
    st.cells = malloc(sizeof(dpcell) * (size_t)st.capcells);
    st.ncells = 0;

    /* antidiagonal 0: the anchor-adjacent corner */
    st.ad[0].lo = 0; st.ad[0].hi = 0; st.ad[0].off = 0;
    st.ad[0].minlive = 0; st.ad[0].maxlive = 0;
    st.cells[0].H = 0; st.cells[0].E = NEG; st.cells[0].F = NEG; st.cells[0].live = 1;
    st.ncells = 1; st.nad = 1;

    int64_t best = 0, bi = 0, bj = 0;
    int64_t cells = 1;

    for (int64_t k = 1; k <= kmax; k++) {
        const adiag *p1 = &st.ad[k - 1];
        const adiag *p2 = k >= 2 ? &st.ad[k - 2] : NULL;
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        if (p1->minlive <= p1->maxlive) { lo = min64(lo, p1->minlive); hi = max64(hi, p1->maxlive + 1); }
        if (p2 && p2->minlive <= p2->maxlive) { lo = min64(lo, p2->minlive + 1); hi = max64(hi, p2->maxlive + 1); }
        if (lo != INT64_MAX) {
            lo = max64(lo, max64(0, k - nB));
            hi = min64(hi, min64(nA, k));
        }
        adiag *cur = &st.ad[k];
        st.nad = k + 1;
        cur->off = st.ncells;
        cur->minlive = INT64_MAX; cur->maxlive = INT64_MIN;
        if (lo == INT64_MAX || lo > hi) {
            cur->lo = 1; cur->hi = 0;                 /* empty range */
        } else {
            cur->lo = lo; cur->hi = hi;
            int64_t n = hi - lo + 1;
            while (st.ncells + n > st.capcells) {
                st.capcells *= 2;
                st.cells = realloc(st.cells, sizeof(dpcell) * (size_t)st.capcells);
            }
            cells += n;
            int64_t thr = best - Y;                  /* best over antidiagonals < k */
            int64_t admax = INT64_MIN, ami = 0;
            for (int64_t i = lo; i <= hi; i++) {
                int64_t j = k - i;
                int64_t E = clampneg(max64(getH(&st, k - 1, i) - oe, getE(&st, k - 1, i) - e));
                int64_t F = clampneg(max64(getH(&st, k - 1, i - 1) - oe, getF(&st, k - 1, i - 1) - e));
                int64_t G = NEG;
                if (i >= 1 && j >= 1)
                    G = clampneg(getH(&st, k - 2, i - 1) + subst(sc, at(A, i - 1), at(B, j - 1)));
                int64_t H = clampneg(max64(G, max64(E, F)));
                dpcell *c = &st.cells[st.ncells + (i - lo)];
                c->H = (int32_t)H; c->E = (int32_t)E; c->F = (int32_t)F;
                c->live = (H >= thr);
                if (c->live) {
                    if (i < cur->minlive) cur->minlive = i;
                    if (i > cur->maxlive) cur->maxlive = i;
                    if (H > admax) { admax = H; ami = i; }
                }
            }
            st.ncells += n;
            if (admax > best) { best = admax; bi = ami; bj = k - ami; }
        }
        /* stop after two consecutive antidiagonals without a live cell */
        int cur_empty = cur->minlive > cur->maxlive;
        int prev_empty = p1->minlive > p1->maxlive;
        if (cur_empty && prev_empty) break;
    }

    res->best = (int32_t)best;
    res->i_end = bi;
    res->j_end = bj;
    res->cells = cells;

    /* traceback from the stored values; in H: diagonal > E > F, in a gap state:
     * open > extend */
    *nops = 0;
    int64_t i = bi, j = bj;
    int state = 0; /* 0 H, 1 E, 2 F */
    while (!(i == 0 && j == 0 && state == 0)) {
        int64_t k = i + j;
        if (state == 0) {
            int64_t h = getH(&st, k, i);
            int64_t g = NEG;
            if (i >= 1 && j >= 1) g = clampneg(getH(&st, k - 2, i - 1) + subst(sc, at(A, i - 1), at(B, j - 1)));
            if (h == g) { emit(ops, nops, opscap, 0); i--; j--; }
            else if (h == getE(&st, k, i)) state = 1;
            else state = 2;
        } else if (state == 1) {
            emit(ops, nops, opscap, 1);
            if (getE(&st, k, i) == getH(&st, k - 1, i) - oe) state = 0;
            j--;
        } else {
            emit(ops, nops, opscap, 2);
            if (getF(&st, k, i) == getH(&st, k - 1, i - 1) - oe) state = 0;
            i--;
        }
    }
    res->n_ops = *nops;
    free(st.ad);
    free(st.cells);
}

int64_t orc_ydrop_half(const uint8_t *A, int64_t nA, const uint8_t *B, int64_t nB,
                       const orc_scoring *sc, orc_half *res, uint8_t *ops, int64_t ops_cap)
{
    seqview va = { A, 1 }, vb = { B, 1 };
    uint8_t *buf = NULL;
    int64_t n = 0, cap = 0;
    ydrop_half(va, nA, vb, nB, sc, res, &buf, &n, &cap);
    for (int64_t x = 0; x < n && x < ops_cap; x++) ops[x] = buf[x];
    free(buf);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Extension of one HSP: the anchor is the HSP's middle column            */
/* (offset (len-1)/2), itself part of the alignment; the two halves run    */
/* the same DP forwards and backwards from the columns next to it.          */
/* ------------------------------------------------------------------------ */
typedef struct { uint8_t *ops; int64_t n, cap; } opvec;

static void push_run(uint32_t **runs, int64_t *n, int64_t *cap, uint8_t op)
{
    if (*n > 0 && ((*runs)[*n - 1] & 3u) == op) { (*runs)[*n - 1] += 4u; return; }
    if (*n == *cap) { *cap = *cap ? 2 * *cap : 64; *runs = realloc(*runs, sizeof(uint32_t) * (size_t)*cap); }
    (*runs)[(*n)++] = (1u << 2) | op;
}

/* Extends the anchor column (ta, qa); fills the alignment and its edit
 * operations as run-length words (len << 2 | op, op 0 M, 1 I, 2 D). */
static void extend_anchor(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
                          int64_t ta, int64_t qa, const orc_scoring *sc,
                          orc_aln *a, uint32_t **runs, int64_t *nruns, int64_t *runcap)
{
    orc_half fw, bw;
    uint8_t *fops = NULL, *bops = NULL;
    int64_t nf = 0, nb = 0, cf = 0, cb = 0;
    seqview fA = { tc + ta + 1, 1 }, fB = { qc + qa + 1, 1 };
    seqview bA = { tc + ta - 1, -1 }, bB = { qc + qa - 1, -1 };
    ydrop_half(fA, nt - ta - 1, fB, nq - qa - 1, sc, &fw, &fops, &nf, &cf);
    ydrop_half(bA, ta, bB, qa, sc, &bw, &bops, &nb, &cb);

    a->score = (int64_t)subst(sc, tc[ta], qc[qa]) + fw.best + bw.best;
    a->t_start = ta - bw.i_end;
    a->t_end = ta + 1 + fw.i_end;
    a->q_start = qa - bw.j_end;
    a->q_end = qa + 1 + fw.j_end;
    a->anchor_t = ta;
    a->anchor_q = qa;
    a->cells = fw.cells + bw.cells;

    *nruns = 0;
    /* backward half: emission order already runs left to right */
    for (int64_t x = 0; x < nb; x++) push_run(runs, nruns, runcap, bops[x]);
    push_run(runs, nruns, runcap, 0);                        /* the anchor column */
    for (int64_t x = nf - 1; x >= 0; x--) push_run(runs, nruns, runcap, fops[x]);
    free(fops);
    free(bops);
}

int64_t orc_extend(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
                   int64_t ta, int64_t qa, const orc_scoring *sc, orc_aln *out,
                   uint32_t *ops, int64_t ops_cap)
{
    uint32_t *runs = NULL;
    int64_t n = 0, cap = 0;
    extend_anchor(tc, nt, qc, nq, ta, qa, sc, out, &runs, &n, &cap);
    for (int64_t x = 0; x < n && x < ops_cap; x++) ops[x] = runs[x];
    out->ops_len = n;
    free(runs);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Committed M columns of one (query, strand) unit, for the anchor test of  */
/* Alg. 1 and Alg. 3: an anchor is covered when it lies on an M column of   */
/* an alignment committed earlier in the same unit.  Each M run is kept as  */
/* (diagonal d = t - q, [t_begin, t_end)) in a hash table chained by d.     */
/* ------------------------------------------------------------------------ */
typedef struct run { int64_t d, tb, te; struct run *next; } run;
#define NBUCKET (1 << 18)
typedef struct { run **bucket; } seglist;

static uint64_t hdiag(int64_t d) { return ((uint64_t)d * 0x9E3779B97F4A7C15ull) >> 46; }

static void seg_init(seglist *s) { s->bucket = calloc(NBUCKET, sizeof(run *)); }
static void seg_free(seglist *s)
{
    for (int64_t b = 0; b < NBUCKET; b++) {
        run *r = s->bucket[b];
        while (r) { run *nx = r->next; free(r); r = nx; }
    }
    free(s->bucket);
}
static int seg_contains(const seglist *s, int64_t t, int64_t q)
{
    int64_t d = t - q;
    for (run *r = s->bucket[hdiag(d)]; r; r = r->next)
        if (r->d == d && r->tb <= t && t < r->te) return 1;
    return 0;
}
static void seg_add_alignment(seglist *s, const orc_aln *a, const uint32_t *runs, int64_t nruns)
{
    int64_t t = a->t_start, q = a->q_start;
    for (int64_t x = 0; x < nruns; x++) {
        int64_t len = runs[x] >> 2;
        int op = runs[x] & 3;
        if (op == 0) {
            run *r = malloc(sizeof(run));
            r->d = t - q; r->tb = t; r->te = t + len;
            uint64_t h = hdiag(r->d);
            r->next = s->bucket[h];
            s->bucket[h] = r;
            t += len; q += len;
        } else if (op == 1) {
            q += len;
        } else {
            t += len;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The commit walk of one (query, strand) unit (units are independent).    */
/*                                                                          */
/* K <= 0, Alg. 1: the HSPs are visited in the given (canonical) order; an  */
/* HSP whose anchor is covered by the commit list is passed over, any other */
/* is extended, and the extension joins the commit list when its score is   */
/* at least the gapped threshold.                                           */
/*                                                                          */
/* K >= 1, Alg. 3: batches of up to K HSPs whose anchors are not covered    */
/* are gathered in order, all of them are extended, and the batch is then   */
/* walked in order again, each extension joining the commit list unless its */
/* anchor has meanwhile become covered (also by a commit of the same batch) */
/* or its score is below the threshold.                                     */
/* ------------------------------------------------------------------------ */
static void aln_push(orc_result *r, const orc_aln *a, const uint32_t *runs, int64_t nruns)
{
    if (r->n_alns == r->cap_alns) {
        r->cap_alns = r->cap_alns ? 2 * r->cap_alns : 64;
        r->alns = realloc(r->alns, sizeof(orc_aln) * (size_t)r->cap_alns);
    }
    while (r->n_ops + nruns > r->cap_ops) {
        r->cap_ops = r->cap_ops ? 2 * r->cap_ops : 1024;
        r->ops = realloc(r->ops, sizeof(uint32_t) * (size_t)r->cap_ops);
    }
    orc_aln *d = &r->alns[r->n_alns++];
    *d = *a;
    d->ops_off = r->n_ops;
    d->ops_len = nruns;
    memcpy(r->ops + r->n_ops, runs, sizeof(uint32_t) * (size_t)nruns);
    r->n_ops += nruns;
}

static int64_t anchor_off(int64_t len) { return (len - 1) / 2; }   /* middle column */

void orc_commit_unit(const uint8_t *tc, int64_t nt, const uint8_t *qc, int64_t nq,
                     const orc_hsp *hsps, int64_t n, const orc_scoring *sc,
                     int64_t K, int32_t query_id, int32_t strand, orc_result *res)
{
    seglist seg;
    seg_init(&seg);
    uint32_t *runs = NULL;
    int64_t nruns = 0, runcap = 0;

    if (K <= 0) {
        for (int64_t j = 0; j < n; j++) {
            int64_t off = anchor_off(hsps[j].len);
            int64_t ta = hsps[j].t0 + off, qa = hsps[j].q0 + off;
            if (seg_contains(&seg, ta, qa)) continue;           /* anchor covered: pass over */
            orc_aln a;
            extend_anchor(tc, nt, qc, nq, ta, qa, sc, &a, &runs, &nruns, &runcap);
            res->n_extensions++;
            res->ext_cells += a.cells;
            if (a.score >= sc->gapped_thresh) {                 /* threshold is inclusive */
                a.query_id = query_id; a.strand = strand;
                aln_push(res, &a, runs, nruns);                 /* into the output */
                seg_add_alignment(&seg, &a, runs, nruns);       /* its M runs now cover */
            }
        }
    } else {
        int64_t kb = K < n ? K : (n > 0 ? n : 1);             /* a batch never exceeds n */
        int64_t *batch = malloc(sizeof(int64_t) * (size_t)kb);
        orc_aln *ext = malloc(sizeof(orc_aln) * (size_t)kb);
        uint32_t **extruns = calloc((size_t)kb, sizeof(uint32_t *));
        int64_t *extn = calloc((size_t)kb, sizeof(int64_t));
        int64_t j = 0;
        while (j < n) {
            int64_t nbatch = 0;
            while (nbatch < kb && j < n) {                      /* gather the batch */
                int64_t off = anchor_off(hsps[j].len);
                if (!seg_contains(&seg, hsps[j].t0 + off, hsps[j].q0 + off)) batch[nbatch++] = j;
                j++;
            }
            for (int64_t b = 0; b < nbatch; b++) {              /* extensions are independent */
                const orc_hsp *h = &hsps[batch[b]];
                int64_t off = anchor_off(h->len);
                int64_t cap = 0;
                extn[b] = 0;
                extend_anchor(tc, nt, qc, nq, h->t0 + off, h->q0 + off, sc, &ext[b],
                              &extruns[b], &extn[b], &cap);
                res->n_extensions++;
                res->ext_cells += ext[b].cells;
            }
            for (int64_t b = 0; b < nbatch; b++) {              /* in-order commit of the batch */
                orc_aln *a = &ext[b];
                if (!seg_contains(&seg, a->anchor_t, a->anchor_q) && a->score >= sc->gapped_thresh) {
                    a->query_id = query_id; a->strand = strand;
                    aln_push(res, a, extruns[b], extn[b]);
                    seg_add_alignment(&seg, a, extruns[b], extn[b]);
                }
                free(extruns[b]);
                extruns[b] = NULL;
            }
        }
        free(batch); free(ext); free(extruns); free(extn);
    }
    free(runs);
    seg_free(&seg);
}

orc_result *orc_result_new(void) { return calloc(1, sizeof(orc_result)); }
void orc_result_free(orc_result *r)
{
    if (!r) return;
    free(r->alns);
    free(r->ops);
    free(r);
}
