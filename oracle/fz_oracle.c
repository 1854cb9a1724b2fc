/*
 * fz_oracle.c -- CPU oracle for the factorization set
 *
 *     Z(n, (g_1..g_d)) = { (a_1..a_d) in N^d : a_1 g_1 + ... + a_d g_d = n }
 *
 * (paper Sec. 1, the definition of the factorization set; generators may come
 * in any order and may repeat, per the footnote to Sec. 1).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct
 * implementation that the GPU library is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the library itself never does, and the two share no code, header,
 * table or helper.  Every function below is single-threaded and written for
 * a reader to check against the paper by eye, not for speed.
 *
 * Contents (each function cites the passage it follows):
 *   fzo_walk           ascending-lex nested loops: the definition written out,
 *                      feeding a count / length-histogram / predicate / store
 *                      consumer (the consumers of Sec. 2)
 *   fzo_dp_count       |Z| as the coefficient of x^n in prod_i 1/(1 - x^{g_i})
 *   fzo_dp_hist        #{a in Z : sum a_i = l} as the coefficient of x^n y^l in
 *                      prod_i 1/(1 - y x^{g_i})
 *   fzo_unrank_dp      the r-th element of Z in ascending lex order, by
 *                      counting completions level by level
 *   fzo_dp_series      |Z(v)| for every v = 0..nmax (the same product, all
 *                      coefficients kept)
 *   fzo_candidate_stream
 *                      the paper's descending candidate stream (first
 *                      candidate of Sec. 3.2.1, successor of Alg. 3.1) with
 *                      the optional modulo skip (Sec. 3.2.4) and bounds
 *                      (Sec. 3.1.2, Sec. 4)
 *
 * Readings of the paper taken here (where it is garbled or silent):
 *   - Alg. 3.1 looks for the coordinate to lower among positions 1..d-1: the
 *     prose excludes the final index, and including it would try to solve
 *     a_{d+1}.
 *   - decrementAndSolve divides by g_{i+1} (the prose once writes g_1).
 *   - Modulo skip: "the order" is the additive order of g_{d-1} modulo g_d,
 *     ord = g_d / gcd(g_{d-1}, g_d).  When a_{d-1} < ord no further valid
 *     tuple has the current prefix; the step then lowers a_{d-1} all the way
 *     to 0 (an invalid candidate that still satisfies Thm. 3.2's hypothesis).
 *   - Counts are exact unsigned 64-bit values; a count that reaches
 *     2^64 - 1 is reported as overflow.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FZO_OK 0
#define FZO_EINVAL (-1)
#define FZO_EOVERFLOW (-2)
#define FZO_ENOMEM (-3)
#define FZO_EINTERNAL (-4)

static uint64_t sat_add(uint64_t x, uint64_t y)
{
    uint64_t s = x + y;
    return (s < x) ? UINT64_MAX : s;
}

static int valid_args(uint64_t n, const uint32_t *g, uint32_t d)
{
    (void)n;
    if (g == NULL || d == 0) return 0;
    for (uint32_t i = 0; i < d; i++)
        if (g[i] == 0) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* The definition written out: ascending lexicographic nested loops.        */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t n;
    const uint32_t *g;
    uint32_t d;
    uint64_t *a;               /* current tuple                              */
    const uint32_t *start;     /* if set: only tuples >=_lex start are taken */
    uint64_t stop_after;       /* stop once this many were taken (0: never)  */
    int stopped;
    /* consumers (Sec. 2: count, predicate, store; plus a length histogram) */
    uint64_t count;
    uint64_t *hist;
    uint64_t nbins;
    int hist_out_of_range;
    uint64_t target_len;
    int found;
    uint32_t *out;
    uint64_t out_cap;
    uint64_t written;
} walk_t;

static void take(walk_t *w)
{
    uint64_t len = 0;
    for (uint32_t i = 0; i < w->d; i++) len += w->a[i];
    w->count++;
    if (w->hist) {
        if (len < w->nbins) w->hist[len]++;
        else w->hist_out_of_range = 1;
    }
    if (len == w->target_len) w->found = 1;
    if (w->out && w->written < w->out_cap) {
        for (uint32_t i = 0; i < w->d; i++)
            w->out[w->written * w->d + i] = (uint32_t)w->a[i];
        w->written++;
    }
    if (w->stop_after && w->count >= w->stop_after) w->stopped = 1;
}

/* Level k (0-based) chooses a_k with rem = n - sum_{j<k} a_j g_j left over.
 * a_k runs upward from 0 (ascending lex order), except that while the prefix
 * still equals start's prefix it runs from start[k].  The last coordinate is
 * not searched: a_d = rem / g_d when g_d divides rem, else there is none. */
static void walk_level(walk_t *w, uint32_t k, uint64_t rem, int on_start)
{
    const uint64_t gk = w->g[k];
    if (w->stopped) return;
    if (k == w->d - 1) {
        if (rem % gk != 0) return;
        w->a[k] = rem / gk;
        if (on_start && w->a[k] < w->start[k]) return;
        take(w);
        return;
    }
    uint64_t lo = on_start ? w->start[k] : 0;
    for (uint64_t t = lo; t * gk <= rem; t++) {
        w->a[k] = t;
        walk_level(w, k + 1, rem - t * gk, on_start && t == lo);
        if (w->stopped) return;
    }
}

/*
 * fzo_walk: visit Z(n,g) in ascending lexicographic order of the caller's
 * coordinate order (Sec. 1 defines Z; Sec. 2 lists the consumers).
 *   start      NULL, or a d-tuple: only elements >=_lex start are visited
 *   stop_after 0, or stop after that many visited elements
 *   count      out: number visited
 *   hist/nbins optional: hist[l] += 1 for each element of length l = sum a_i
 *              (*hist_oor set to 1 if some length is >= nbins)
 *   target_len / found: *found = 1 if some visited element has length target
 *   out/out_cap optional: the first out_cap visited elements, row-major [.][d]
 *   written    out: rows written
 */
int fzo_walk(uint64_t n, const uint32_t *g, uint32_t d, const uint32_t *start,
             uint64_t stop_after, uint64_t *count, uint64_t *hist,
             uint64_t nbins, int *hist_oor, uint64_t target_len, int *found,
             uint32_t *out, uint64_t out_cap, uint64_t *written)
{
    if (!valid_args(n, g, d) || count == NULL) return FZO_EINVAL;
    walk_t w;
    memset(&w, 0, sizeof w);
    w.n = n;
    w.g = g;
    w.d = d;
    w.a = (uint64_t *)calloc(d, sizeof(uint64_t));
    if (!w.a) return FZO_ENOMEM;
    w.start = start;
    w.stop_after = stop_after;
    w.hist = hist;
    w.nbins = nbins;
    w.target_len = target_len;
    w.out = out;
    w.out_cap = out ? out_cap : 0;
    if (hist) memset(hist, 0, nbins * sizeof(uint64_t));
    walk_level(&w, 0, n, start != NULL);
    *count = w.count;
    if (hist_oor) *hist_oor = w.hist_out_of_range;
    if (found) *found = w.found;
    if (written) *written = w.written;
    free(w.a);
    return FZO_OK;
}

/* ------------------------------------------------------------------------ */
/* Generating-function counts (the dynamic-programming view, Sec. 1).       */
/* ------------------------------------------------------------------------ */

/* |Z(n,g)| = [x^n] prod_i 1/(1 - x^{g_i}).  Multiplying the series by one
 * factor 1/(1 - x^g) is c[v] += c[v - g] for v ascending.  Saturating
 * arithmetic: a coefficient that reaches 2^64 - 1 stays there, so the answer
 * is exact unless it is reported as overflow. */
int fzo_dp_count(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count)
{
    if (!valid_args(n, g, d) || count == NULL) return FZO_EINVAL;
    uint64_t *c = (uint64_t *)calloc(n + 1, sizeof(uint64_t));
    if (!c) return FZO_ENOMEM;
    c[0] = 1;
    for (uint32_t i = 0; i < d; i++)
        for (uint64_t v = g[i]; v <= n; v++)
            c[v] = sat_add(c[v], c[v - g[i]]);
    uint64_t r = c[n];
    free(c);
    if (r == UINT64_MAX) return FZO_EOVERFLOW;
    *count = r;
    return FZO_OK;
}

/* The whole series: series[v] = |Z(v,g)| for v = 0..nmax (UINT64_MAX marks a
 * coefficient that overflowed).  Same multiplication as fzo_dp_count. */
int fzo_dp_series(uint64_t nmax, const uint32_t *g, uint32_t d, uint64_t *series)
{
    if (!valid_args(nmax, g, d) || series == NULL) return FZO_EINVAL;
    memset(series, 0, (nmax + 1) * sizeof(uint64_t));
    series[0] = 1;
    for (uint32_t i = 0; i < d; i++)
        for (uint64_t v = g[i]; v <= nmax; v++)
            series[v] = sat_add(series[v], series[v - g[i]]);
    return FZO_OK;
}

/* hist[l] = [x^n y^l] prod_i 1/(1 - y x^{g_i}) for l < nbins.  One factor is
 * c[v][l] += c[v - g][l - 1] for v ascending.  Needs (n+1)*nbins words. */
int fzo_dp_hist(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *hist,
                uint64_t nbins)
{
    if (!valid_args(n, g, d) || hist == NULL || nbins == 0) return FZO_EINVAL;
    uint64_t cells = (n + 1) * nbins;
    if (nbins != 0 && cells / nbins != n + 1) return FZO_ENOMEM;
    uint64_t *c = (uint64_t *)calloc(cells, sizeof(uint64_t));
    if (!c) return FZO_ENOMEM;
    c[0] = 1; /* the empty product: v = 0, length 0 */
    for (uint32_t i = 0; i < d; i++)
        for (uint64_t v = g[i]; v <= n; v++)
            for (uint64_t l = 1; l < nbins; l++)
                c[v * nbins + l] =
                    sat_add(c[v * nbins + l], c[(v - g[i]) * nbins + l - 1]);
    int rc = FZO_OK;
    for (uint64_t l = 0; l < nbins; l++) {
        hist[l] = c[n * nbins + l];
        if (hist[l] == UINT64_MAX) rc = FZO_EOVERFLOW;
    }
    free(c);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Unranking: the r-th element (0-based) of Z in ascending lex order.       */
/* ------------------------------------------------------------------------ */

/* T[k][v] = number of (a_k..a_d) >= 0 with sum_{j>=k} a_j g_j = v, i.e. the
 * count of completions of a prefix that left v over.  T[d][v] = [v == 0] and
 * T[k][v] = sum_{t>=0} T[k+1][v - t g_k], computed as the same coin-change
 * recurrence T[k][v] = T[k+1][v] + T[k][v - g_k].  Then level by level the
 * completions with a_k = 0, 1, 2, ... are skipped until r falls inside one. */
int fzo_unrank_dp(uint64_t n, const uint32_t *g, uint32_t d, uint64_t r,
                  uint32_t *out)
{
    if (!valid_args(n, g, d) || out == NULL) return FZO_EINVAL;
    uint64_t *T = (uint64_t *)calloc((uint64_t)(d + 1) * (n + 1), sizeof(uint64_t));
    if (!T) return FZO_ENOMEM;
#define TT(k, v) T[(uint64_t)(k) * (n + 1) + (v)]
    TT(d, 0) = 1;
    for (int k = (int)d - 1; k >= 0; k--)
        for (uint64_t v = 0; v <= n; v++)
            TT(k, v) = sat_add(TT(k + 1, v), v >= g[k] ? TT(k, v - g[k]) : 0);
    int rc = FZO_OK;
    if (TT(0, n) == UINT64_MAX) rc = FZO_EOVERFLOW;
    else if (r >= TT(0, n)) rc = FZO_EINVAL;
    else {
        uint64_t v = n;
        for (uint32_t k = 0; k < d; k++) {
            uint64_t t = 0;
            for (;;) {
                uint64_t c = TT(k + 1, v - t * g[k]);
                if (r < c) break;
                r -= c;
                t++;
                if (t * g[k] > v) { rc = FZO_EINTERNAL; break; }
            }
            if (rc) break;
            out[k] = (uint32_t)t;
            v -= t * g[k];
        }
    }
#undef TT
    free(T);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The paper's candidate stream (Sec. 3), descending lexicographic order.   */
/* ------------------------------------------------------------------------ */

/* ParallelLexicographicState (Sec. 3.1.2): element n, generators g, bound b,
 * previousCandidate a, wasValid, endOfStream.  Coordinates are stored 0-based
 * (a[0] is the paper's a_1). */
typedef struct {
    uint64_t n;
    const uint32_t *g;
    uint32_t d;
    uint64_t *a;
    const uint64_t *b;
    int was_valid;
    int end_of_stream;
} fzo_state;

static uint64_t phi(const fzo_state *s)
{
    uint64_t t = 0;
    for (uint32_t i = 0; i < s->d; i++) t += s->a[i] * s->g[i];
    return t;
}

static int lex_le(const uint64_t *x, const uint64_t *y, uint32_t d)
{
    for (uint32_t i = 0; i < d; i++) {
        if (x[i] < y[i]) return 1;
        if (x[i] > y[i]) return 0;
    }
    return 1;
}

static uint64_t gcd64(uint64_t x, uint64_t y)
{
    while (y) {
        uint64_t t = x % y;
        x = y;
        y = t;
    }
    return x;
}

/* First candidate (Sec. 3.2.1): (x, 0, ..., 0) with x = ceil(n / g_1); it is
 * a factorization exactly when g_1 divides n. */
static void first_candidate(fzo_state *s)
{
    for (uint32_t i = 0; i < s->d; i++) s->a[i] = 0;
    uint64_t x = (s->n + s->g[0] - 1) / s->g[0];
    s->a[0] = x;
    s->was_valid = (x * s->g[0] == s->n);
    s->end_of_stream = 0;
}

/* Successor in the descending candidate stream: Alg. 3.1 (nextCandidate),
 * with the modulo skip of Sec. 3.2.4 when use_modulo is set, written here
 * from the order it walks rather than as the printed listing.
 *
 * In descending lex order, the candidate after a = (a_1..a_d) keeps the
 * longest prefix it can: let k be the last position before d whose
 * coordinate is positive (none: the stream is over).  Everything after k
 * restarts from its largest admissible value, so the successor is
 *     (a_1, .., a_{k-1}, a_k - step, c, 0, .., 0),
 * where c is the least value for which the candidate reaches n or more,
 * c = ceil(p / g_{k+1}) for the residual p = n - sum_{j<=k} a_j g_j; the new
 * candidate is a factorization exactly when g_{k+1} divides p.  The step is
 * one, except after a factorization whose last changed position is d-1:
 * then the next factorization with the same a_1..a_{d-2} has a_{d-1} lower by
 * the additive order of g_{d-1} modulo g_d (Sec. 3.2.4), and when a_{d-1} is
 * below that order none is left, so a_{d-1} drops to 0.  The stream also
 * ends at the first candidate that is <=_lex the bound (Sec. 3.1.2).
 * Returns FZO_EINTERNAL if the residual is not positive, which Thm. 3.2's
 * hypothesis rules out. */
static int next_candidate(fzo_state *s, int use_modulo)
{
    const uint32_t d = s->d;
    uint64_t *a = s->a;
    if (s->end_of_stream) return FZO_OK;

    /* the last positive coordinate among positions 1..d-1 (0-based: k-1) */
    uint32_t k = d - 1;
    while (k > 0 && a[k - 1] == 0) k--;
    if (k == 0) {
        s->end_of_stream = 1;
        return FZO_OK;
    }
    uint32_t pos = k - 1; /* 0-based index of the coordinate that is lowered */

    uint64_t step = 1;
    if (use_modulo && pos == d - 2 && s->was_valid) {
        uint64_t order = s->g[d - 1] / gcd64(s->g[d - 2], s->g[d - 1]);
        step = a[pos] < order ? a[pos] : order;
    }
    a[pos] -= step;
    for (uint32_t j = pos + 1; j < d; j++) a[j] = 0;

    uint64_t used = phi(s);
    if (used >= s->n) return FZO_EINTERNAL;
    uint64_t residual = s->n - used;
    uint64_t gnext = s->g[pos + 1];
    a[pos + 1] = (residual + gnext - 1) / gnext;      /* ceiling division */
    s->was_valid = (a[pos + 1] * gnext == residual);

    if (lex_le(a, s->b, d)) s->end_of_stream = 1;
    return FZO_OK;
}

/*
 * fzo_candidate_stream: run the candidate stream of one worker and collect
 * what a consumer of Alg. 3.1's output would see.
 *   start      NULL: begin at the first candidate (Sec. 3.2.1);
 *              else a d-tuple used as previousCandidate (it must satisfy
 *              Thm. 3.2's hypothesis; it is not itself reported)
 *   bound      NULL: (0,...,0), the whole set (Sec. 3.1.2); else a d-tuple
 *   use_modulo apply the Sec. 3.2.4 skip
 *   valid/cap  optional: the valid candidates in stream order (descending),
 *              row-major [.][d]
 *   n_valid    out: number of valid candidates reported
 *   n_cand     out: number of candidates produced (first one included)
 *   max_coord  optional out, length d: largest value each coordinate took
 *              in any candidate (for the bound of Thm. 3.3)
 * A candidate that ends the stream by reaching the bound is not reported
 * (it belongs to the worker that owns the bound).
 */
int fzo_candidate_stream(uint64_t n, const uint32_t *g, uint32_t d,
                         const uint32_t *start, const uint32_t *bound,
                         int use_modulo, uint32_t *valid, uint64_t cap,
                         uint64_t *n_valid, uint64_t *n_cand,
                         uint64_t *max_coord)
{
    if (!valid_args(n, g, d) || n_valid == NULL || n_cand == NULL)
        return FZO_EINVAL;
    uint64_t *a = (uint64_t *)calloc(d, sizeof(uint64_t));
    uint64_t *b = (uint64_t *)calloc(d, sizeof(uint64_t));
    if (!a || !b) {
        free(a);
        free(b);
        return FZO_ENOMEM;
    }
    if (bound)
        for (uint32_t i = 0; i < d; i++) b[i] = bound[i];
    fzo_state s = {n, g, d, a, b, 0, 0};
    uint64_t nv = 0, nc = 0;
    int rc = FZO_OK;
    if (max_coord)
        for (uint32_t i = 0; i < d; i++) max_coord[i] = 0;
#define REPORT()                                                        \
    do {                                                                \
        if (max_coord)                                                  \
            for (uint32_t q = 0; q < d; q++)                            \
                if (a[q] > max_coord[q]) max_coord[q] = a[q];           \
        if (s.was_valid) {                                              \
            if (valid && nv < cap)                                      \
                for (uint32_t q = 0; q < d; q++)                        \
                    valid[nv * d + q] = (uint32_t)a[q];                 \
            nv++;                                                       \
        }                                                               \
    } while (0)
    if (start == NULL) {
        first_candidate(&s);
        nc++;
        if (!(bound && lex_le(a, b, d))) REPORT();
        else s.end_of_stream = 1;
    } else {
        for (uint32_t i = 0; i < d; i++) a[i] = start[i];
        uint64_t ph = phi(&s);
        s.was_valid = (ph == n);
        s.end_of_stream = 0;
    }
    while (!s.end_of_stream) {
        rc = next_candidate(&s, use_modulo);
        if (rc) break;
        if (s.end_of_stream) break;
        nc++;
        REPORT();
    }
#undef REPORT
    *n_valid = nv;
    *n_cand = nc;
    free(a);
    free(b);
    return rc;
}
