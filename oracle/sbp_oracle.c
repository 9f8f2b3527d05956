/*
 * sbp_oracle.c -- plain, slow, single-threaded FP64 reference of stochastic
 * block partitioning (SBP) on the degree-corrected blockmodel.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * Every function follows a passage of Wanye, Gleyzer, Kao, Feng, "Exact
 * Distributed Stochastic Block Partitioning" (arXiv 2305.18663):
 *   - blockmodel matrix M and block degrees ............ Sec. II-A
 *   - log-likelihood L(G|B) .............................. Eq. 1
 *   - description length DL and h(x) ..................... Eq. 2
 *   - block merge phase .................................. Alg. 1
 *   - MCMC phase (Metropolis-Hastings vertex moves) ...... Alg. 2
 *   - asynchronous-Gibbs batches (moves evaluated against
 *     a stale blockmodel, then all applied) ............. Sec. II-B, Sec. III-B, Alg. 5
 *   - golden-ratio search over the block count ........... Sec. II-B
 *   - sparse change vector for the DL difference ......... Sec. III-A (c)
 *   - merge tracking by pointers (union-find) ............ Sec. III-A (d)
 * Points the paper leaves open (proposal law, temperature, Hastings term,
 * tie-breaks, stop rule, golden steps, random numbers) follow the written
 * readings listed in the repository's design notes; each is restated where
 * it is used below.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011), implemented here from that paper.
 *
 * Parity: pinned by closed forms (C = 1, C = N), the literal Eq. 1, full
 * recomputation of every delta, brute-force minima on tiny graphs, exact
 * enumeration of the proposal law and exact detailed balance; see tests/.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* f(x) = x ln x with f(0) = 0 (Eq. 1 and Eq. 2 in entropy form)        */
/* ------------------------------------------------------------------ */
static double xlogx(double x) { return x > 0.0 ? x * log(x) : 0.0; }

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011, Sec. 3.2 / Table 2)               */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Four 64-bit words from two Philox blocks with counters
 * (a, b, base + i, tag), i = 0, 1; key = (seed low, seed high). */
void orc_words(uint64_t seed, uint32_t a, uint32_t b, uint32_t base, uint32_t tag, uint64_t W[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t i = 0; i < 2; ++i) {
        uint32_t ctr[4] = {a, b, base + i, tag};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        W[2 * i] = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        W[2 * i + 1] = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
    }
}

/* Uniform index in [0, n) from a 64-bit word: floor(W * n / 2^64). */
static int64_t draw_index(uint64_t W, uint64_t n)
{
    return (int64_t)(((unsigned __int128)W * (unsigned __int128)n) >> 64);
}

/* ------------------------------------------------------------------ */
/* Blockmodel: M as a sorted coordinate list with row and column index  */
/* (the "hashmap rows plus transpose" of Sec. III-A (a,b), kept plain)  */
/* ------------------------------------------------------------------ */
typedef struct {
    int C;
    int64_t nnz;
    int64_t *rptr; int *rcol; int64_t *rval;  /* rows: entries (a, b) sorted by b */
    int64_t *cptr; int *crow; int64_t *cval;  /* columns: entries (a, b) sorted by a */
    int64_t *dout, *din;                      /* block out/in degrees */
    int64_t E;
    int N;
} obm;

static int cmp_i64(const void *x, const void *y)
{
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

static void obm_free(obm *m)
{
    free(m->rptr); free(m->rcol); free(m->rval);
    free(m->cptr); free(m->crow); free(m->cval);
    free(m->dout); free(m->din);
    memset(m, 0, sizeof *m);
}

/* M_ab = number of edges (u, w) with b(u) = a and b(w) = b (Sec. II-A);
 * d_a^out = sum_b M_ab, d_b^in = sum_a M_ab (Eq. 1). */
static int obm_build(obm *m, int n, const int *out_ptr, const int *out_idx, const int *lab, int C)
{
    memset(m, 0, sizeof *m);
    int64_t E = out_ptr[n];
    m->C = C; m->E = E; m->N = n;
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    if (!keys) return -1;
    for (int u = 0; u < n; ++u)
        for (int64_t j = out_ptr[u]; j < out_ptr[u + 1]; ++j)
            keys[j] = (int64_t)lab[u] * C + lab[out_idx[j]];
    qsort(keys, (size_t)E, sizeof(int64_t), cmp_i64);
    int64_t nnz = 0;
    for (int64_t j = 0; j < E; ++j)
        if (j == 0 || keys[j] != keys[j - 1]) ++nnz;
    m->nnz = nnz;
    m->rptr = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
    m->cptr = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
    m->rcol = (int *)malloc(sizeof(int) * (size_t)(nnz + 1));
    m->crow = (int *)malloc(sizeof(int) * (size_t)(nnz + 1));
    m->rval = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz + 1));
    m->cval = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz + 1));
    m->dout = (int64_t *)calloc((size_t)C, sizeof(int64_t));
    m->din = (int64_t *)calloc((size_t)C, sizeof(int64_t));
    if (!m->rptr || !m->cptr || !m->rcol || !m->crow || !m->rval || !m->cval || !m->dout || !m->din) {
        free(keys); obm_free(m); return -1;
    }
    int64_t k = -1;
    for (int64_t j = 0; j < E; ++j) {
        if (j == 0 || keys[j] != keys[j - 1]) {
            ++k;
            m->rcol[k] = (int)(keys[j] % C);
            m->rval[k] = 0;
            m->rptr[keys[j] / C + 1]++;
        }
        m->rval[k]++;
    }
    for (int a = 0; a < C; ++a) m->rptr[a + 1] += m->rptr[a];
    /* columns: re-key the entries by (b, a) */
    int64_t *ck = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz + 1));
    if (!ck) { free(keys); obm_free(m); return -1; }
    for (int a = 0; a < C; ++a)
        for (int64_t j = m->rptr[a]; j < m->rptr[a + 1]; ++j)
            ck[j] = (int64_t)m->rcol[j] * C + a;
    qsort(ck, (size_t)nnz, sizeof(int64_t), cmp_i64);
    for (int64_t j = 0; j < nnz; ++j) {
        int b = (int)(ck[j] / C), a = (int)(ck[j] % C);
        m->crow[j] = a;
        m->cptr[b + 1]++;
    }
    for (int b = 0; b < C; ++b) m->cptr[b + 1] += m->cptr[b];
    free(ck);
    free(keys);
    /* values of the column list by lookup in the row list */
    for (int b = 0; b < C; ++b)
        for (int64_t j = m->cptr[b]; j < m->cptr[b + 1]; ++j) {
            int a = m->crow[j];
            int64_t lo = m->rptr[a], hi = m->rptr[a + 1];
            while (lo < hi) { int64_t mid = (lo + hi) / 2; if (m->rcol[mid] < b) lo = mid + 1; else hi = mid; }
            m->cval[j] = m->rval[lo];
        }
    for (int a = 0; a < C; ++a)
        for (int64_t j = m->rptr[a]; j < m->rptr[a + 1]; ++j) {
            m->dout[a] += m->rval[j];
            m->din[m->rcol[j]] += m->rval[j];
        }
    return 0;
}

static int64_t obm_get(const obm *m, int a, int b)
{
    int64_t lo = m->rptr[a], hi = m->rptr[a + 1];
    while (lo < hi) { int64_t mid = (lo + hi) / 2; if (m->rcol[mid] < b) lo = mid + 1; else hi = mid; }
    return (lo < m->rptr[a + 1] && m->rcol[lo] == b) ? m->rval[lo] : 0;
}

/* ------------------------------------------------------------------ */
/* Description length (Eq. 1 and Eq. 2)                                 */
/*   L  = sum_ab M_ab ln(M_ab / (dout_a din_b))                          */
/*      = sum_ab f(M_ab) - sum_a f(dout_a) - sum_b f(din_b)              */
/*   DL = E h(C^2/E) + N ln C - L,  E h(C^2/E) = f(E+C^2) - f(E) - f(C^2) */
/* Summation order: model terms, then f(M) in ascending (a, b), then     */
/* out-degrees, then in-degrees.                                         */
/* ------------------------------------------------------------------ */
static double model_terms(int64_t E, int64_t N, int64_t C)
{
    double e = (double)E, c2 = (double)C * (double)C;
    return xlogx(e + c2) - xlogx(e) - xlogx(c2) + (double)N * log((double)C);
}

static double obm_dl(const obm *m)
{
    double L = 0.0;
    for (int64_t j = 0; j < m->nnz; ++j) L += xlogx((double)m->rval[j]);
    for (int a = 0; a < m->C; ++a) L -= xlogx((double)m->dout[a]);
    for (int b = 0; b < m->C; ++b) L -= xlogx((double)m->din[b]);
    return model_terms(m->E, m->N, m->C) - L;
}

/* Exported: build M and return it as sorted COO plus degrees and DL. */
int orc_build_blockmodel(int n, const int *out_ptr, const int *out_idx, const int *lab, int C,
                         int64_t *nnz_out, int *rows, int *cols, int64_t *vals,
                         int64_t *dout, int64_t *din, double *dl)
{
    for (int v = 0; v < n; ++v)
        if (lab[v] < 0 || lab[v] >= C) return -3;
    obm m;
    if (obm_build(&m, n, out_ptr, out_idx, lab, C)) return -1;
    *nnz_out = m.nnz;
    for (int a = 0; a < C; ++a)
        for (int64_t j = m.rptr[a]; j < m.rptr[a + 1]; ++j) {
            if (rows) rows[j] = a;
            if (cols) cols[j] = m.rcol[j];
            if (vals) vals[j] = m.rval[j];
        }
    if (dout) memcpy(dout, m.dout, sizeof(int64_t) * (size_t)C);
    if (din) memcpy(din, m.din, sizeof(int64_t) * (size_t)C);
    if (dl) *dl = obm_dl(&m);
    obm_free(&m);
    return 0;
}

double orc_description_length(int n, const int *out_ptr, const int *out_idx, const int *lab, int C)
{
    obm m;
    if (obm_build(&m, n, out_ptr, out_idx, lab, C)) return NAN;
    double d = obm_dl(&m);
    obm_free(&m);
    return d;
}

/* ------------------------------------------------------------------ */
/* Proposal: draw from e_t. in ascending block order, where              */
/*   e_ts = M_ts + M_st (s != t),  e_tt = 2 M_tt,  sum_s e_ts = d_t.      */
/* Returns the smallest s whose running sum exceeds x (0 <= x < d_t).   */
/* ------------------------------------------------------------------ */
static int neighbour_block_draw(const obm *m, int t, int64_t x)
{
    int64_t i = m->rptr[t], ie = m->rptr[t + 1];
    int64_t j = m->cptr[t], je = m->cptr[t + 1];
    int64_t run = 0;
    while (i < ie || j < je) {
        int si = i < ie ? m->rcol[i] : m->C;
        int sj = j < je ? m->crow[j] : m->C;
        int s = si < sj ? si : sj;
        if (si == s) run += m->rval[i++];
        if (sj == s) run += m->cval[j++];
        if (run > x) return s;
    }
    return -1; /* unreachable when x < d_t */
}

/* ------------------------------------------------------------------ */
/* One vertex move evaluated against a fixed blockmodel (Alg. 2 body).  */
/* ------------------------------------------------------------------ */
typedef struct {
    int s;          /* proposed block */
    double dS;      /* change of DL if v moves r -> s (C fixed) */
    double lnH;     /* ln q(s->r) - ln q(r->s) */
    double z;       /* -beta dS + lnH */
    double lnu;     /* ln of the accept uniform */
    int accept;
} omove;

typedef struct { int a, b; int64_t d; } ochg;

static int cmp_chg(const void *x, const void *y)
{
    const ochg *p = (const ochg *)x, *q = (const ochg *)y;
    if (p->a != q->a) return (p->a > q->a) - (p->a < q->a);
    return (p->b > q->b) - (p->b < q->b);
}

static int cmp_int(const void *x, const void *y)
{
    int a = *(const int *)x, b = *(const int *)y;
    return (a > b) - (a < b);
}

/* post-move entry: M_ab plus its aggregated change (list sorted by (a, b)) */
static int64_t post_get(const obm *m, const ochg *chg, int nchg, int a, int b)
{
    int lo = 0, hi = nchg;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (chg[mid].a < a || (chg[mid].a == a && chg[mid].b < b)) lo = mid + 1; else hi = mid;
    }
    int64_t d = (lo < nchg && chg[lo].a == a && chg[lo].b == b) ? chg[lo].d : 0;
    return obm_get(m, a, b) + d;
}

static void eval_vertex(const obm *m, int n, const int *out_ptr, const int *out_idx,
                        const int *in_ptr, const int *in_idx, const int *lab, int v,
                        const uint64_t W[4], double beta, int64_t eps, omove *mv)
{
    (void)n;
    const int C = m->C;
    const int r = lab[v];
    const int64_t kout = out_ptr[v + 1] - out_ptr[v];
    const int64_t kin = in_ptr[v + 1] - in_ptr[v];
    const int64_t k = kout + kin;
    memset(mv, 0, sizeof *mv);

    /* proposal (reading of "propose new community", Alg. 2): pick a random
     * edge end of v, let t be the block at its other end, then with
     * probability eps*C/(d_t + eps*C) a uniform block, else a block drawn
     * from e_t. -- the directed neighbour-block proposal of Peixoto 2014. */
    int s;
    if (k == 0) {
        s = (int)draw_index(W[2], (uint64_t)C);
    } else {
        int64_t j = draw_index(W[0], (uint64_t)k);
        int u = j < kout ? out_idx[out_ptr[v] + j] : in_idx[in_ptr[v] + (j - kout)];
        int t = lab[u];
        int64_t dt = m->dout[t] + m->din[t];
        if (draw_index(W[1], (uint64_t)(dt + eps * C)) < eps * C)
            s = (int)draw_index(W[2], (uint64_t)C);
        else
            s = neighbour_block_draw(m, t, draw_index(W[2], (uint64_t)dt));
    }
    mv->s = s;
    mv->lnu = log(((double)(W[3] >> 11) + 0.5) * (1.0 / 9007199254740992.0));
    if (s == r) { mv->accept = 0; return; }

    /* sparse vector of changes (Sec. III-A (c)): every entry of M touched by
     * moving v from r to s, with its net count change. */
    int64_t nends = k;
    ochg *chg = (ochg *)malloc(sizeof(ochg) * (size_t)(4 * nends + 4));
    int nchg = 0;
    int64_t self = 0;
    for (int64_t j = out_ptr[v]; j < out_ptr[v + 1]; ++j) {
        int u = out_idx[j];
        if (u == v) { ++self; continue; }
        int t = lab[u];
        chg[nchg++] = (ochg){r, t, -1};
        chg[nchg++] = (ochg){s, t, +1};
    }
    for (int64_t j = in_ptr[v]; j < in_ptr[v + 1]; ++j) {
        int u = in_idx[j];
        if (u == v) continue;
        int t = lab[u];
        chg[nchg++] = (ochg){t, r, -1};
        chg[nchg++] = (ochg){t, s, +1};
    }
    if (self) {
        chg[nchg++] = (ochg){r, r, -self};
        chg[nchg++] = (ochg){s, s, +self};
    }
    qsort(chg, (size_t)nchg, sizeof(ochg), cmp_chg);
    int w = 0;
    for (int i = 0; i < nchg; ++i) {
        if (w > 0 && chg[w - 1].a == chg[i].a && chg[w - 1].b == chg[i].b) chg[w - 1].d += chg[i].d;
        else chg[w++] = chg[i];
    }
    nchg = w;

    /* change of L (Eq. 1 in f form) over the touched entries and degrees */
    double dL = 0.0;
    for (int i = 0; i < nchg; ++i) {
        int64_t before = obm_get(m, chg[i].a, chg[i].b);
        dL += xlogx((double)(before + chg[i].d)) - xlogx((double)before);
    }
    dL -= xlogx((double)(m->dout[r] - kout)) - xlogx((double)m->dout[r]);
    dL -= xlogx((double)(m->dout[s] + kout)) - xlogx((double)m->dout[s]);
    dL -= xlogx((double)(m->din[r] - kin)) - xlogx((double)m->din[r]);
    dL -= xlogx((double)(m->din[s] + kin)) - xlogx((double)m->din[s]);
    mv->dS = -dL; /* C is unchanged by a vertex move, so dDL = -dL (Eq. 2) */

    /* Hastings term: q(r->s) = sum_t (k_t/k) (e_ts + eps)/(d_t + eps C) on
     * the current blockmodel; q(s->r) the same law after the move. */
    double lnH = 0.0;
    if (k > 0) {
        int *nb = (int *)malloc(sizeof(int) * (size_t)(nends + 1));
        int64_t cnt = 0;
        for (int64_t j = out_ptr[v]; j < out_ptr[v + 1]; ++j) nb[cnt++] = out_idx[j];
        for (int64_t j = in_ptr[v]; j < in_ptr[v + 1]; ++j) nb[cnt++] = in_idx[j];
        /* blocks of the other ends before (self ends sit in r) and after (in s) */
        int *tb = (int *)malloc(sizeof(int) * (size_t)(nends + 1));
        int *ta = (int *)malloc(sizeof(int) * (size_t)(nends + 1));
        for (int64_t j = 0; j < cnt; ++j) {
            tb[j] = nb[j] == v ? r : lab[nb[j]];
            ta[j] = nb[j] == v ? s : lab[nb[j]];
        }
        qsort(tb, (size_t)cnt, sizeof(int), cmp_int);
        qsort(ta, (size_t)cnt, sizeof(int), cmp_int);
        double qf = 0.0, qr = 0.0;
        for (int64_t j = 0; j < cnt;) {
            int t = tb[j];
            int64_t kt = 0;
            while (j < cnt && tb[j] == t) { ++kt; ++j; }
            int64_t ets = t == s ? 2 * obm_get(m, s, s) : obm_get(m, t, s) + obm_get(m, s, t);
            int64_t dt = m->dout[t] + m->din[t];
            qf += (double)kt * ((double)(ets + eps) / (double)(dt + eps * C));
        }
        for (int64_t j = 0; j < cnt;) {
            int t = ta[j];
            int64_t kt = 0;
            while (j < cnt && ta[j] == t) { ++kt; ++j; }
            int64_t etr = t == r ? 2 * post_get(m, chg, nchg, r, r)
                                 : post_get(m, chg, nchg, t, r) + post_get(m, chg, nchg, r, t);
            int64_t dt = m->dout[t] + m->din[t] + (t == r ? -k : 0) + (t == s ? k : 0);
            qr += (double)kt * ((double)(etr + eps) / (double)(dt + eps * C));
        }
        lnH = log(qr) - log(qf);
        free(nb); free(tb); free(ta);
    }
    free(chg);
    mv->lnH = lnH;
    mv->z = -beta * mv->dS + lnH;
    mv->accept = mv->lnu < mv->z;
}

/* Exported single-move evaluation (for exact enumeration and detailed
 * balance checks): the blockmodel is built from lab, the words are given. */
int orc_eval_move(int n, const int *out_ptr, const int *out_idx, const int *in_ptr, const int *in_idx,
                  const int *lab, int C, int v, const uint64_t W[4], double beta, int64_t eps,
                  int *s, double *dS, double *lnH, double *lnu, int *accept)
{
    obm m;
    if (obm_build(&m, n, out_ptr, out_idx, lab, C)) return -1;
    omove mv;
    eval_vertex(&m, n, out_ptr, out_idx, in_ptr, in_idx, lab, v, W, beta, eps, &mv);
    *s = mv.s; *dS = mv.dS; *lnH = mv.lnH; *lnu = mv.lnu; *accept = mv.accept;
    obm_free(&m);
    return 0;
}

/* ------------------------------------------------------------------ */
/* One sweep of the MCMC phase (Alg. 2 inner loop) in the hybrid form    */
/* of Sec. II-B: the n_hubs vertices of highest degree (out + in edge    */
/* ends; ties by smaller id) move first, one at a time in that order,    */
/* each evaluated against the assignment left by the previous one and    */
/* applied at once (sequential Metropolis-Hastings).  The other vertices */
/* then move in asynchronous-Gibbs batches (Sec. II-B / Alg. 5): batch   */
/* j = {v : v mod n_batches = j, v not a hub}, evaluated against the     */
/* blockmodel at the batch start, then all its accepted moves applied.   */
/* n_hubs = 0 is the plain asynchronous sweep; n_batches = n is          */
/* sequential Alg. 2.  (The paper does not fix the order of the two      */
/* parts or the hub count; both are readings, see the design notes.)    */
/* Words for v: counter (v, sweep, 0|1, 0).                              */
/* force (nullable): force[v] >= 0 replaces the accept decision of v.    */
/* stats: [proposals, self proposals, accepted, forced]                  */
/* ------------------------------------------------------------------ */
static int *g_deg_sort;  /* degrees for the hub order comparator */
static int hub_cmp(const void *x, const void *y)
{
    const int a = *(const int *)x, b = *(const int *)y;
    if (g_deg_sort[a] != g_deg_sort[b]) return g_deg_sort[a] > g_deg_sort[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

/* The first n_hubs vertices in descending degree, ties by smaller id. */
int orc_hub_order(int n, const int *out_ptr, const int *in_ptr, int n_hubs, int *order)
{
    if (n_hubs < 0 || n_hubs > n) return -1;
    int *deg = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *all = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int v = 0; v < n; ++v) {
        deg[v] = (out_ptr[v + 1] - out_ptr[v]) + (in_ptr[v + 1] - in_ptr[v]);
        all[v] = v;
    }
    g_deg_sort = deg;
    qsort(all, (size_t)n, sizeof(int), hub_cmp);
    memcpy(order, all, sizeof(int) * (size_t)n_hubs);
    free(deg); free(all);
    return 0;
}

static void record_move(const omove *mv, int v, const int *lab, const int8_t *force, int64_t *st, double *sacc,
                        int *prop, double *dS, double *lnH, double *z, double *lnu, int8_t *acc, int *a_out)
{
    int a = mv->accept;
    if (force && force[v] >= 0) { if (force[v] != a) st[3]++; a = force[v]; }
    st[0]++;
    if (mv->s == lab[v]) { st[1]++; a = 0; }
    if (a) { st[2]++; *sacc += mv->dS; }
    if (prop) prop[v] = mv->s;
    if (dS) dS[v] = mv->dS;
    if (lnH) lnH[v] = mv->lnH;
    if (z) z[v] = mv->z;
    if (lnu) lnu[v] = mv->lnu;
    if (acc) acc[v] = (int8_t)a;
    *a_out = a;
}

int orc_nodal_sweep_h(int n, const int *out_ptr, const int *out_idx, const int *in_ptr, const int *in_idx,
                      int *lab, int C, uint64_t seed, uint32_t sweep, double beta, int64_t eps,
                      int n_batches, int n_hubs, int *prop, double *dS, double *lnH, double *z, double *lnu,
                      int8_t *acc, const int8_t *force, int64_t *stats, double *sum_dS)
{
    if (n_batches < 1) n_batches = 1;
    if (n_batches > n) n_batches = n;
    if (n_hubs < 0 || n_hubs > n) return -1;
    int64_t st[4] = {0, 0, 0, 0};
    double sacc = 0.0;
    int *news = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int8_t *acc_local = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
    int8_t *hub = (int8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int *order = (int *)malloc(sizeof(int) * (size_t)(n_hubs > 0 ? n_hubs : 1));
    orc_hub_order(n, out_ptr, in_ptr, n_hubs, order);
    /* the hubs, one at a time against the current assignment */
    for (int i = 0; i < n_hubs; ++i) {
        const int v = order[i];
        hub[v] = 1;
        obm m;
        if (obm_build(&m, n, out_ptr, out_idx, lab, C)) { free(news); free(acc_local); free(hub); free(order); return -1; }
        uint64_t W[4];
        orc_words(seed, (uint32_t)v, sweep, 0, 0, W);
        omove mv;
        eval_vertex(&m, n, out_ptr, out_idx, in_ptr, in_idx, lab, v, W, beta, eps, &mv);
        int a;
        record_move(&mv, v, lab, force, st, &sacc, prop, dS, lnH, z, lnu, acc, &a);
        if (a) lab[v] = mv.s;
        obm_free(&m);
    }
    /* the rest in asynchronous batches */
    for (int j = 0; j < n_batches; ++j) {
        obm m;
        if (obm_build(&m, n, out_ptr, out_idx, lab, C)) { free(news); free(acc_local); free(hub); free(order); return -1; }
        for (int v = j; v < n; v += n_batches) {
            if (hub[v]) continue;
            uint64_t W[4];
            orc_words(seed, (uint32_t)v, sweep, 0, 0, W);
            omove mv;
            eval_vertex(&m, n, out_ptr, out_idx, in_ptr, in_idx, lab, v, W, beta, eps, &mv);
            int a;
            record_move(&mv, v, lab, force, st, &sacc, prop, dS, lnH, z, lnu, acc, &a);
            news[v] = mv.s; acc_local[v] = (int8_t)a;
        }
        for (int v = j; v < n; v += n_batches)
            if (!hub[v] && acc_local[v]) lab[v] = news[v];
        obm_free(&m);
    }
    free(news); free(acc_local); free(hub); free(order);
    if (stats) memcpy(stats, st, sizeof st);
    if (sum_dS) *sum_dS = sacc;
    return 0;
}

int orc_nodal_sweep(int n, const int *out_ptr, const int *out_idx, const int *in_ptr, const int *in_idx,
                    int *lab, int C, uint64_t seed, uint32_t sweep, double beta, int64_t eps,
                    int n_batches, int *prop, double *dS, double *lnH, double *z, double *lnu,
                    int8_t *acc, const int8_t *force, int64_t *stats, double *sum_dS)
{
    return orc_nodal_sweep_h(n, out_ptr, out_idx, in_ptr, in_idx, lab, C, seed, sweep, beta, eps, n_batches, 0,
                             prop, dS, lnH, z, lnu, acc, force, stats, sum_dS);
}

/* ------------------------------------------------------------------ */
/* Block merge scoring (Alg. 1, proposal loop).                         */
/* For block c and j < x, words from counter (c, phase, 2j|2j+1, 1).     */
/* Proposal: if d_c = 0, uniform over the other C-1 blocks; otherwise t  */
/* is drawn from e_c., then with probability eps*C/(d_t+eps*C) a uniform  */
/* block != c, else a block from e_t.; c' = c is an invalid proposal.    */
/* dS_local = -(change of L when c and c' become one block); the full    */
/* change of DL adds the model-term change for C -> C-1.  Candidates are */
/* compared on floor(dS_local * 2^20): differences below 2^-20 nats are  */
/* treated as ties and the first proposal is kept.                       */
/* ------------------------------------------------------------------ */
static int64_t rank_key(double x)
{
    if (!(x < 1e300)) return INT64_MAX;
    return (int64_t)floor(x * 1048576.0);
}

static double merge_delta_L(const obm *m, int c, int cp)
{
    /* rows c and c' combine into one; then columns; then the 2x2 corner */
    double dL = 0.0;
    int64_t i = m->rptr[c], ie = m->rptr[c + 1], j = m->rptr[cp], je = m->rptr[cp + 1];
    while (i < ie || j < je) {
        int ti = i < ie ? m->rcol[i] : m->C, tj = j < je ? m->rcol[j] : m->C;
        int t = ti < tj ? ti : tj;
        int64_t x = 0, y = 0;
        if (ti == t) x = m->rval[i++];
        if (tj == t) y = m->rval[j++];
        if (t == c || t == cp) continue;
        dL += xlogx((double)(x + y)) - xlogx((double)x) - xlogx((double)y);
    }
    i = m->cptr[c]; ie = m->cptr[c + 1]; j = m->cptr[cp]; je = m->cptr[cp + 1];
    while (i < ie || j < je) {
        int ti = i < ie ? m->crow[i] : m->C, tj = j < je ? m->crow[j] : m->C;
        int t = ti < tj ? ti : tj;
        int64_t x = 0, y = 0;
        if (ti == t) x = m->cval[i++];
        if (tj == t) y = m->cval[j++];
        if (t == c || t == cp) continue;
        dL += xlogx((double)(x + y)) - xlogx((double)x) - xlogx((double)y);
    }
    int64_t a = obm_get(m, c, c), b = obm_get(m, c, cp), e = obm_get(m, cp, c), g = obm_get(m, cp, cp);
    dL += xlogx((double)(a + b + e + g)) - xlogx((double)a) - xlogx((double)b) - xlogx((double)e) - xlogx((double)g);
    dL -= xlogx((double)(m->dout[c] + m->dout[cp])) - xlogx((double)m->dout[c]) - xlogx((double)m->dout[cp]);
    dL -= xlogx((double)(m->din[c] + m->din[cp])) - xlogx((double)m->din[c]) - xlogx((double)m->din[cp]);
    return dL;
}

/* One merge proposal for block c from the words W (Alg. 1, "propose a new
 * community c' to merge with c"; the law is a reading, the paper gives none):
 * with d_c = 0 a uniform block among the C-1 others, idx(W2, C-1) skipping c;
 * otherwise t is the block of a random edge end of c, drawn from e_c. with
 * idx(W0, d_c); then a uniform block among the C-1 others when
 * idx(W1, d_t + eps C) < eps C, else a block drawn from e_t. with idx(W2, d_t).
 * The result may be c itself (an invalid proposal). */
static int merge_propose(const obm *m, int c, const uint64_t W[4], int64_t eps)
{
    const int C = m->C;
    int64_t dc = m->dout[c] + m->din[c];
    if (dc == 0) {
        int64_t kk = draw_index(W[2], (uint64_t)(C - 1));
        return (int)(kk + (kk >= c));
    }
    int t = neighbour_block_draw(m, c, draw_index(W[0], (uint64_t)dc));
    int64_t dt = m->dout[t] + m->din[t];
    if (draw_index(W[1], (uint64_t)(dt + eps * C)) < eps * C) {
        int64_t kk = draw_index(W[2], (uint64_t)(C - 1));
        return (int)(kk + (kk >= c));
    }
    return neighbour_block_draw(m, t, draw_index(W[2], (uint64_t)dt));
}

/* The x proposals of every block (words from counter (c, phase, 2j|2j+1, 1)
 * for j < x).  A proposal of c itself is invalid and still counts toward x.
 * The valid candidate with the smallest floor(dS_local 2^20) is kept, the
 * first on ties; without one, partner = -1 and dS = +inf. */
static void merge_scores_on(const obm *m, uint64_t seed, uint32_t phase, int x, int64_t eps,
                            int *partner, double *dS, double *dS_local)
{
    const int C = m->C;
    const double offset = model_terms(m->E, m->N, C - 1) - model_terms(m->E, m->N, C);
    for (int c = 0; c < C; ++c) {
        int best = -1;
        double best_local = INFINITY;
        for (int j = 0; j < x && C > 1; ++j) {
            uint64_t W[4];
            orc_words(seed, (uint32_t)c, phase, (uint32_t)(2 * j), 1, W);
            int cp = merge_propose(m, c, W, eps);
            if (cp == c) continue;
            double local = -merge_delta_L(m, c, cp);
            if (rank_key(local) < rank_key(best_local)) { best = cp; best_local = local; }
        }
        partner[c] = best;
        dS_local[c] = best < 0 ? INFINITY : best_local;
        dS[c] = best < 0 ? INFINITY : best_local + offset;
    }
}

/* Exported: the partner block one set of words proposes for c (may be c). */
int orc_merge_propose(int n, const int *out_ptr, const int *out_idx, const int *lab, int C, int c,
                      const uint64_t W[4], int64_t eps)
{
    if (c < 0 || c >= C || C < 2) return -1;
    obm m;
    if (obm_build(&m, n, out_ptr, out_idx, lab, C)) return -1;
    int cp = merge_propose(&m, c, W, eps);
    obm_free(&m);
    return cp;
}

/* Exported: full DL change and its local part for merging c and cp. */
int orc_merge_delta(int n, const int *out_ptr, const int *out_idx, const int *lab, int C, int c, int cp,
                    double *dS, double *dS_local)
{
    if (c < 0 || cp < 0 || c >= C || cp >= C || c == cp || C < 2) return -1;
    obm m;
    if (obm_build(&m, n, out_ptr, out_idx, lab, C)) return -1;
    *dS_local = -merge_delta_L(&m, c, cp);
    *dS = *dS_local + model_terms(m.E, m.N, C - 1) - model_terms(m.E, m.N, C);
    obm_free(&m);
    return 0;
}

int orc_merge_scores(int n, const int *out_ptr, const int *out_idx, const int *lab, int C,
                     uint64_t seed, uint32_t phase, int x, int64_t eps,
                     int *partner, double *dS, double *dS_local)
{
    obm m;
    if (obm_build(&m, n, out_ptr, out_idx, lab, C)) return -1;
    merge_scores_on(&m, seed, phase, x, eps, partner, dS, dS_local);
    obm_free(&m);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Merge application (Alg. 1, "sort best_merges, pop and merge until the */
/* count is reached", with pointer-based tracking of Sec. III-A (d)).    */
/* Candidates in ascending (floor(dS_local*2^20), c); merging joins the  */
/* set of c into the set of its partner; pairs already joined or without */
/* a partner are skipped.  New labels number the merged groups in the   */
/* ascending order of their smallest member block (a canonical order     */
/* that does not depend on the order of the unions).  Returns the new   */
/* block count.                                                          */
/* ------------------------------------------------------------------ */
static int uf_find(int *parent, int a)
{
    while (parent[a] != a) { parent[a] = parent[parent[a]]; a = parent[a]; }
    return a;
}

typedef struct { int64_t key; int c; } ocand;

static int cmp_cand(const void *x, const void *y)
{
    const ocand *p = (const ocand *)x, *q = (const ocand *)y;
    if (p->key != q->key) return (p->key > q->key) - (p->key < q->key);
    return (p->c > q->c) - (p->c < q->c);
}

int orc_merge_apply(int C, const int *partner, const double *dS_local, int n_merges, int *map)
{
    ocand *cand = (ocand *)malloc(sizeof(ocand) * (size_t)C);
    int *parent = (int *)malloc(sizeof(int) * (size_t)C);
    for (int c = 0; c < C; ++c) { cand[c].key = rank_key(dS_local[c]); cand[c].c = c; parent[c] = c; }
    qsort(cand, (size_t)C, sizeof(ocand), cmp_cand);
    int done = 0;
    for (int i = 0; i < C && done < n_merges; ++i) {
        int c = cand[i].c, p = partner[c];
        if (p < 0) continue;
        int a = uf_find(parent, c), b = uf_find(parent, p);
        if (a == b) continue;
        parent[a] = b;
        ++done;
    }
    /* smallest member of each group, then groups numbered in that order */
    int *low = (int *)malloc(sizeof(int) * (size_t)C);
    for (int c = 0; c < C; ++c) low[c] = C;
    for (int c = 0; c < C; ++c) {
        int root = uf_find(parent, c);
        if (c < low[root]) low[root] = c;
    }
    int next = 0;
    int *rank = (int *)malloc(sizeof(int) * (size_t)C);
    for (int c = 0; c < C; ++c) rank[c] = (low[uf_find(parent, c)] == c) ? next++ : -1;
    for (int c = 0; c < C; ++c) map[c] = rank[low[uf_find(parent, c)]];
    free(low); free(rank); free(parent); free(cand);
    return next;
}

/* Drop empty labels, keeping the order of the rest; returns the count. */
static int compact_labels(int n, int *lab, int C)
{
    int *map = (int *)malloc(sizeof(int) * (size_t)(C > 0 ? C : 1));
    for (int c = 0; c < C; ++c) map[c] = 0;
    for (int v = 0; v < n; ++v) map[lab[v]] = 1;
    int next = 0;
    for (int c = 0; c < C; ++c) map[c] = map[c] ? next++ : -1;
    for (int v = 0; v < n; ++v) lab[v] = map[lab[v]];
    free(map);
    return next;
}

int orc_compact(int n, int *lab, int C) { return compact_labels(n, lab, C); }

/* ------------------------------------------------------------------ */
/* Golden-ratio search over the block count (Sec. II-B; the steps after */
/* the bracket exists are a reading: integer golden-section search).    */
/* Slots 0 = hi, 1 = mid, 2 = lo hold (C, DL) with C_hi > C_mid > C_lo  */
/* and DL_mid the least stored DL.                                      */
/* ------------------------------------------------------------------ */
/* Inserts result (Cr, dlr).  A result better than mid becomes mid and
 * the old mid moves to hi when Cr < C_mid, else to lo; a result that is not
 * better replaces lo when Cr < C_mid, else hi.  The first result becomes
 * mid.  Returns the slot written; *displaced (nullable) receives the slot
 * the old mid moved to, or -1. */
int orc_golden_insert(int C[3], double dl[3], int used[3], int Cr, double dlr, int *displaced)
{
    int to = 1, moved = -1;
    if (!used[1]) {
        to = 1;
    } else if (dlr < dl[1]) {
        moved = Cr < C[1] ? 0 : 2;
        C[moved] = C[1]; dl[moved] = dl[1]; used[moved] = 1;
        to = 1;
    } else {
        to = Cr < C[1] ? 2 : 0;
    }
    C[to] = Cr; dl[to] = dlr; used[to] = 1;
    if (displaced) *displaced = moved;
    return to;
}

/* Next block count to try.  Before a bracket exists (no lo): halve from mid,
 * target C_mid - floor(C_mid merge_rate) (Alg. 1, "until the number of
 * communities is halved").  With a bracket, the larger of the segments
 * (C_hi - C_mid) and (C_mid - C_lo) is split 0.382 of its length away from
 * mid: upper: C_mid + max(1, round(0.381966 (C_hi - C_mid))), below C_hi,
 * merged down from hi; lower: C_lo + max(1, round(0.618034 (C_mid - C_lo))),
 * below C_mid, merged down from mid.  Returns the start slot (0 or 1) and
 * writes *target, or returns -1 when the search is over: C_hi - C_lo <= 2,
 * C_mid - C_lo <= 1 without hi, or no merge left before the bracket. */
int orc_golden_next(const int C[3], const int used[3], double merge_rate, int *target)
{
    if (!used[2]) {
        int merges = (int)floor(C[1] * merge_rate);
        if (merges < 1) return -1;
        *target = C[1] - merges;
        return 1;
    }
    int upper = used[0] ? C[0] - C[1] : 0;
    int lower = C[1] - C[2];
    if (used[0] ? (C[0] - C[2] <= 2) : (lower <= 1)) return -1;
    if (used[0] && upper >= lower) {
        int step = (int)floor(0.381966 * upper + 0.5);
        if (step < 1) step = 1;
        int t = C[1] + step;
        *target = t > C[0] - 1 ? C[0] - 1 : t;
        return 0;
    }
    int step = (int)floor(0.618034 * lower + 0.5);
    if (step < 1) step = 1;
    int t = C[2] + step;
    *target = t > C[1] - 1 ? C[1] - 1 : t;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Whole method (Sec. II-B): agglomerative alternation of block merges  */
/* and MCMC, with the golden-ratio search over the block count.         */
/* An iteration merges the start assignment down to the target count    */
/* (Alg. 1), runs the MCMC phase at that count (Alg. 2; blocks it        */
/* empties stay as empty labels, so C in Eq. 2 is the count the merge   */
/* phase produced) and stores (C, DL, assignment) in the golden triple.  */
/* The returned assignment is the best stored one with its empty labels */
/* dropped, and its DL is recomputed at the non-empty count.            */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    double beta;
    int64_t eps;
    int merge_proposals;
    int max_sweeps;
    double t_pre, t_post;
    double merge_rate;
    int n_batches;
    int max_iters;
    int n_hubs;  /* hybrid sweeps (R21): hubs moved one at a time first; 0 = none */
} opart_params;

/* One MCMC phase (Alg. 2 outer loop) at C blocks: sweeps until
 * |DL_prev - DL| < t DL after a sweep, or max_sweeps sweeps; the sweep index
 * in the random-number counter continues from *sweep_ctr.  Returns the
 * number of sweeps and writes the final DL. */
static int mcmc_phase(int n, const int *out_ptr, const int *out_idx, const int *in_ptr, const int *in_idx,
                      int *lab, int C, const opart_params *p, double tol, uint32_t *sweep_ctr, double *dl_out)
{
    double dl_prev = orc_description_length(n, out_ptr, out_idx, lab, C);
    double dl = dl_prev;
    int sweeps = 0;
    while (sweeps < p->max_sweeps) {
        orc_nodal_sweep_h(n, out_ptr, out_idx, in_ptr, in_idx, lab, C, p->seed, (*sweep_ctr)++, p->beta, p->eps,
                          p->n_batches, p->n_hubs < n ? p->n_hubs : n, NULL, NULL, NULL, NULL, NULL, NULL, NULL,
                          NULL, NULL);
        ++sweeps;
        dl = orc_description_length(n, out_ptr, out_idx, lab, C);
        int stop = fabs(dl_prev - dl) < tol * dl;
        dl_prev = dl;
        if (stop) break;
    }
    *dl_out = dl;
    return sweeps;
}

/* trace row per iteration: [C_start, C_target, C_merged, sweeps, C_stored] as int64, and DL */
int orc_partition(int n, const int *out_ptr, const int *out_idx, const int *in_ptr, const int *in_idx,
                  const int *lab_in, int C_in, const opart_params *p,
                  int *lab_out, int *C_out, double *dl_out,
                  int64_t *trace, double *trace_dl, int trace_cap, int *n_iters)
{
    if (n < 1) return -1;
    int *lab = (int *)malloc(sizeof(int) * (size_t)n);
    int C;
    if (lab_in) {
        for (int v = 0; v < n; ++v) {
            if (lab_in[v] < 0 || lab_in[v] >= C_in) { free(lab); return -3; }
            lab[v] = lab_in[v];
        }
        C = compact_labels(n, lab, C_in);
    } else {
        for (int v = 0; v < n; ++v) lab[v] = v;
        C = n;
    }
    /* golden triple: counts, DLs and assignments of slots hi, mid, lo */
    int gC[3] = {0, 0, 0}, gused[3] = {0, 0, 0};
    double gdl[3] = {0, 0, 0};
    int *glab[3];
    for (int k = 0; k < 3; ++k) glab[k] = (int *)malloc(sizeof(int) * (size_t)n);
    uint32_t sweep_ctr = 0, phase_ctr = 0;
    int iters = 0;

    /* store the assignment in lab as the result (Cr, dlr) */
#define GOLDEN_STORE(CR, DLR) do { int from_ = -1; \
        int to_ = orc_golden_insert(gC, gdl, gused, (CR), (DLR), &from_); \
        if (from_ >= 0) { int *t_ = glab[from_]; glab[from_] = glab[1]; glab[1] = t_; } \
        memcpy(glab[to_], lab, sizeof(int) * (size_t)n); } while (0)

    GOLDEN_STORE(C, orc_description_length(n, out_ptr, out_idx, lab, C));

    int *map = (int *)malloc(sizeof(int) * (size_t)n);
    int *partner = (int *)malloc(sizeof(int) * (size_t)n);
    double *dS = (double *)malloc(sizeof(double) * (size_t)n);
    double *dSl = (double *)malloc(sizeof(double) * (size_t)n);

    while (iters < p->max_iters) {
        int target;
        int from = orc_golden_next(gC, gused, p->merge_rate, &target);
        if (from < 0) break;
        int C0 = gC[from];
        memcpy(lab, glab[from], sizeof(int) * (size_t)n);

        /* block merge phase (Alg. 1) */
        orc_merge_scores(n, out_ptr, out_idx, lab, C0, p->seed, phase_ctr++, p->merge_proposals, p->eps,
                         partner, dS, dSl);
        int C1 = orc_merge_apply(C0, partner, dSl, C0 - target, map);
        for (int v = 0; v < n; ++v) lab[v] = map[lab[v]];

        /* MCMC phase (Alg. 2) at C1 blocks */
        double dlR;
        int sweeps = mcmc_phase(n, out_ptr, out_idx, in_ptr, in_idx, lab, C1, p,
                                gused[2] ? p->t_post : p->t_pre, &sweep_ctr, &dlR);
        if (trace && iters < trace_cap) {
            trace[5 * iters + 0] = C0; trace[5 * iters + 1] = target; trace[5 * iters + 2] = C1;
            trace[5 * iters + 3] = sweeps; trace[5 * iters + 4] = C1;
            if (trace_dl) trace_dl[iters] = dlR;
        }
        ++iters;
        GOLDEN_STORE(C1, dlR);
    }
#undef GOLDEN_STORE
    /* the best result without its empty labels */
    memcpy(lab_out, glab[1], sizeof(int) * (size_t)n);
    int Cf = compact_labels(n, lab_out, gC[1]);
    *C_out = Cf;
    *dl_out = orc_description_length(n, out_ptr, out_idx, lab_out, Cf);
    if (n_iters) *n_iters = iters;
    for (int k = 0; k < 3; ++k) free(glab[k]);
    free(lab); free(map); free(partner); free(dS); free(dSl);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Divide-and-conquer SBP (Sec. II-C, Alg. 3), one process.              */
/* Readings (the paper describes the steps, not every rule):             */
/*  - subgraph r of s keeps the vertices v with v mod s = r and the      */
/*    edges whose two ends it keeps ("round robin sample"); kept         */
/*    vertices are renumbered in ascending order;                        */
/*  - subgraph r is partitioned by the whole method with seed + 1 + r;   */
/*  - combining results P1, P2 ("merge B2 communities into B1            */
/*    communities"): on the graph induced by the vertices of both, with  */
/*    P2's labels after P1's, every community c of P2 joins the          */
/*    community c1 of P1 whose merge with c changes DL least (compared   */
/*    on floor(dS_local 2^20) as in Alg. 1, the lowest c1 on ties), all  */
/*    choices taken against the blockmodel before any of them is        */
/*    applied;                                                           */
/*  - rounds pair results (0,1), (2,3), ...; an odd last one passes on;  */
/*    rounds repeat while more than 4 results remain;                    */
/*  - the remaining results are concatenated (labels of result k after   */
/*    those of results 0..k-1) and the whole method continues on the     */
/*    full graph from that assignment with the caller's seed.            */
/* ------------------------------------------------------------------ */

/* Induced subgraph of the vertices with keep[v] != 0: ids renumbered in
 * ascending order (sub_id[v] = new id or -1), CSR then CSC; sizes in
 * *n_sub, *e_sub.  Output arrays sized for the whole graph. */
int orc_induced(int n, const int *out_ptr, const int *out_idx, const int *in_ptr, const int *in_idx,
                const unsigned char *keep, int *sub_id, int *s_out_ptr, int *s_out_idx, int *s_in_ptr,
                int *s_in_idx, int *n_sub, int *e_sub)
{
    int k = 0;
    for (int v = 0; v < n; ++v) sub_id[v] = keep[v] ? k++ : -1;
    int e = 0, ei = 0;
    s_out_ptr[0] = 0;
    s_in_ptr[0] = 0;
    for (int v = 0; v < n; ++v) {
        if (!keep[v]) continue;
        for (int j = out_ptr[v]; j < out_ptr[v + 1]; ++j)
            if (keep[out_idx[j]]) s_out_idx[e++] = sub_id[out_idx[j]];
        for (int j = in_ptr[v]; j < in_ptr[v + 1]; ++j)
            if (keep[in_idx[j]]) s_in_idx[ei++] = sub_id[in_idx[j]];
        s_out_ptr[sub_id[v] + 1] = e;
        s_in_ptr[sub_id[v] + 1] = ei;
    }
    *n_sub = k;
    *e_sub = e;
    return e == ei ? 0 : -1;
}

/* The merge choice of combining: lab holds P1's labels [0, C1) and P2's
 * [C1, C1 + C2) on the induced graph; best[c2] = the chosen community of P1
 * for community C1 + c2 (or -1 when C1 = 0). */
int orc_combine_choice(int n, const int *out_ptr, const int *out_idx, const int *lab, int C1, int C2, int *best)
{
    obm m;
    if (obm_build(&m, n, out_ptr, out_idx, lab, C1 + C2)) return -1;
    for (int c2 = 0; c2 < C2; ++c2) {
        int b = -1;
        int64_t bkey = INT64_MAX;
        for (int c1 = 0; c1 < C1; ++c1) {
            int64_t key = rank_key(-merge_delta_L(&m, C1 + c2, c1));
            if (b < 0 || key < bkey) { b = c1; bkey = key; }
        }
        best[c2] = b;
    }
    obm_free(&m);
    return 0;
}

typedef struct { int nv; int *vid; int *lab; int C; } opiece;  /* global ids ascending */

int orc_dcsbp(int n, const int *out_ptr, const int *out_idx, const int *in_ptr, const int *in_idx, int s,
              const opart_params *p, int *lab_out, int *C_out, double *dl_out, int *sub_C)
{
    if (n < 1 || s < 1 || s > n) return -1;
    const int e = out_ptr[n];
    unsigned char *keep = (unsigned char *)malloc((size_t)n);
    int *sid = (int *)malloc(sizeof(int) * (size_t)n);
    int *sop = (int *)malloc(sizeof(int) * ((size_t)n + 1)), *sip = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *soi = (int *)malloc(sizeof(int) * ((size_t)e + 1)), *sii = (int *)malloc(sizeof(int) * ((size_t)e + 1));
    int *slab = (int *)malloc(sizeof(int) * (size_t)n);
    opiece *R = (opiece *)calloc((size_t)s, sizeof(opiece));
    int nR = s, rc = 0;
    /* 1: every subgraph partitioned on its own */
    for (int r = 0; r < s && !rc; ++r) {
        for (int v = 0; v < n; ++v) keep[v] = (v % s) == r;
        int ns, es;
        if ((rc = orc_induced(n, out_ptr, out_idx, in_ptr, in_idx, keep, sid, sop, soi, sip, sii, &ns, &es))) break;
        opart_params q = *p;
        q.seed = p->seed + 1 + (uint64_t)r;
        int C;
        double dl;
        if ((rc = orc_partition(ns, sop, soi, sip, sii, NULL, 0, &q, slab, &C, &dl, NULL, NULL, 0, NULL))) break;
        R[r].nv = ns;
        R[r].vid = (int *)malloc(sizeof(int) * (size_t)ns);
        R[r].lab = (int *)malloc(sizeof(int) * (size_t)ns);
        for (int v = 0, i = 0; v < n; ++v)
            if (keep[v]) { R[r].vid[i] = v; R[r].lab[i] = slab[i]; ++i; }
        R[r].C = C;
        if (sub_C) sub_C[r] = C;
    }
    /* 2: pairwise combination while more than 4 results remain */
    int *glab = (int *)malloc(sizeof(int) * (size_t)n);
    while (!rc && nR > 4) {
        int k = 0;
        for (int i = 0; i < nR; i += 2) {
            if (i + 1 == nR) { R[k++] = R[i]; break; }
            opiece *a = &R[i], *b = &R[i + 1];
            memset(keep, 0, (size_t)n);
            for (int j = 0; j < a->nv; ++j) { keep[a->vid[j]] = 1; glab[a->vid[j]] = a->lab[j]; }
            for (int j = 0; j < b->nv; ++j) { keep[b->vid[j]] = 1; glab[b->vid[j]] = a->C + b->lab[j]; }
            int ns, es;
            if ((rc = orc_induced(n, out_ptr, out_idx, in_ptr, in_idx, keep, sid, sop, soi, sip, sii, &ns, &es))) break;
            for (int v = 0; v < n; ++v)
                if (keep[v]) slab[sid[v]] = glab[v];
            int *best = (int *)malloc(sizeof(int) * ((size_t)b->C + 1));
            if ((rc = orc_combine_choice(ns, sop, soi, slab, a->C, b->C, best))) { free(best); break; }
            opiece m;
            m.nv = ns;
            m.vid = (int *)malloc(sizeof(int) * (size_t)ns);
            m.lab = (int *)malloc(sizeof(int) * (size_t)ns);
            for (int v = 0; v < n; ++v) {
                if (!keep[v]) continue;
                const int x = slab[sid[v]];
                m.vid[sid[v]] = v;
                m.lab[sid[v]] = x < a->C ? x : best[x - a->C];
            }
            m.C = compact_labels(ns, m.lab, a->C);
            free(best);
            free(a->vid); free(a->lab); free(b->vid); free(b->lab);
            R[k++] = m;
        }
        nR = k;
    }
    /* 3: concatenation, then the whole method on the full graph */
    if (!rc) {
        int off = 0;
        for (int i = 0; i < nR; ++i) {
            for (int j = 0; j < R[i].nv; ++j) glab[R[i].vid[j]] = off + R[i].lab[j];
            off += R[i].C;
        }
        rc = orc_partition(n, out_ptr, out_idx, in_ptr, in_idx, glab, off, p, lab_out, C_out, dl_out, NULL, NULL,
                           0, NULL);
    }
    for (int i = 0; i < nR; ++i) { free(R[i].vid); free(R[i].lab); }
    free(R); free(glab); free(keep); free(sid); free(sop); free(sip); free(soi); free(sii); free(slab);
    return rc;
}
