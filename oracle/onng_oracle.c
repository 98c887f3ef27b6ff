/*
 * Plain CPU oracle (see onng_oracle.h).  TEST INFRASTRUCTURE ONLY: this file is
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the product path, and shares no code with it.
 *
 * The code follows the paper's algorithms step by step, with the readings
 * listed below; it is written for clarity, not speed.
 *
 *   R1  Algorithm 2's loop guard is read "p <= e_o or p <= e_i".
 *   R2  Seeds are de-duplicated, counted as distance computations, marked
 *       visited and offered to R one by one through the R-update rule of
 *       Algorithm 1; S starts as all seeds.
 *   R4  Every argmin/argmax uses the total order (distance, node id).
 *   R5  The range test on squared L2 uses thr = r * f with f = fp32((1+eps)^2)
 *       (eps scales the Euclidean radius); on cosine distance f = fp32(1+eps).
 *       On u8 data the product is an fp32 multiply.
 *   R6  e_p is an integer chosen by the caller; UINT32_MAX means unlimited.
 *       p advances on every scanned edge, visited or not.
 *   R10 Algorithm 3 takes nodes in ascending (|N(G_t, x)|, x); its guard
 *       "N(G_e, o) < e_o" compares the list's size.
 *   R11 AdjustPath visits nodes in ascending id and sees its own additions
 *       immediately.
 *   R12 HasPath keeps the strict "<" on the edge lengths.
 *   R17 Edge lengths are the distances stored in the kNN rows; a reverse edge
 *       takes the length from the row it came from.
 */
#include "onng_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Codecs                                                                     */
/* ------------------------------------------------------------------------- */

/* Exact value of a code in a binary floating format with `eb` exponent bits,
 * `mb` mantissa bits and bias `bias`.  fn_nan: e4m3fn has no infinities and
 * only S.1111.111 is NaN. */
static double decode_format(uint32_t code, int eb, int mb, int bias, int fn_nan)
{
    uint32_t sign = (code >> (eb + mb)) & 1u;
    uint32_t e = (code >> mb) & ((1u << eb) - 1u);
    uint32_t m = code & ((1u << mb) - 1u);
    double v;
    if (fn_nan) {
        if (e == (1u << eb) - 1u && m == (1u << mb) - 1u)
            return NAN;
    } else if (e == (1u << eb) - 1u) {
        v = m ? NAN : INFINITY;
        return sign ? -v : v;
    }
    if (e == 0)
        v = ldexp((double)m, 1 - bias - mb);                 /* subnormal */
    else
        v = ldexp((double)((1u << mb) | m), (int)e - bias - mb);
    return sign ? -v : v;
}

double or_decode(int32_t dtype, uint32_t code)
{
    switch (dtype) {
    case OR_U8: return (double)(code & 0xffu);
    case OR_F32: { float f; memcpy(&f, &code, 4); return (double)f; }
    case OR_F16: return decode_format(code & 0xffffu, 5, 10, 15, 0);
    case OR_BF16: return decode_format(code & 0xffffu, 8, 7, 127, 0);
    case OR_FP8: return decode_format(code & 0xffu, 4, 3, 7, 1);
    }
    return NAN;
}

/* Round |x| (finite, > 0) to the format, nearest-even.  Returns the rounded
 * magnitude; the caller packs it.  emin = 1 - bias. */
static double round_to_format(double a, int mb, int bias)
{
    int ex;
    frexp(a, &ex);                  /* a = f * 2^ex, f in [0.5, 1) */
    int e = ex - 1;                 /* a in [2^e, 2^(e+1)) */
    int emin = 1 - bias;
    if (e < emin)
        e = emin;                   /* subnormal range: fixed quantum */
    double q = ldexp(1.0, e - mb);  /* spacing of representable values */
    double n = a / q;               /* exact: power-of-two scaling */
    double r = nearbyint(n);        /* default rounding mode: nearest-even */
    return r * q;
}

static uint32_t pack_format(double mag, uint32_t sign, int eb, int mb, int bias)
{
    if (mag == 0.0)
        return sign << (eb + mb);
    int ex;
    frexp(mag, &ex);
    int e = ex - 1;
    int emin = 1 - bias;
    uint32_t efield, mfield;
    if (e < emin) {
        efield = 0;
        mfield = (uint32_t)(mag / ldexp(1.0, emin - mb));
    } else {
        efield = (uint32_t)(e + bias);
        mfield = (uint32_t)(mag / ldexp(1.0, e - mb)) - (1u << mb);
    }
    return (sign << (eb + mb)) | (efield << mb) | mfield;
}

static uint32_t encode_ieee(float x, int eb, int mb, int bias)
{
    uint32_t bits; memcpy(&bits, &x, 4);
    uint32_t sign = bits >> 31;
    uint32_t emax_field = (1u << eb) - 1u;
    if (isnan(x))
        return (sign << (eb + mb)) | (emax_field << mb) | (1u << (mb - 1));
    double a = fabs((double)x);
    if (isinf(x))
        return (sign << (eb + mb)) | (emax_field << mb);
    double mag = round_to_format(a, mb, bias);
    double maxf = ldexp((double)((2u << mb) - 1u), (int)(emax_field - 1) - bias - mb);
    if (mag > maxf)                  /* rounded past the largest finite value */
        return (sign << (eb + mb)) | (emax_field << mb);
    return pack_format(mag, sign, eb, mb, bias);
}

uint32_t or_encode_f16(float x) { return encode_ieee(x, 5, 10, 15); }
uint32_t or_encode_bf16(float x) { return encode_ieee(x, 8, 7, 127); }

uint32_t or_encode_fp8(float x)
{
    uint32_t bits; memcpy(&bits, &x, 4);
    uint32_t sign = bits >> 31;
    if (isnan(x))
        return (sign << 7) | 0x7fu;
    double a = fabs((double)x);
    const double maxf = 448.0;
    double mag = isinf(x) ? maxf : round_to_format(a, 3, 7);
    if (mag > maxf)
        mag = maxf;                  /* saturate */
    return pack_format(mag, sign, 4, 3, 7);
}

int or_encode_rows(const float *src, int64_t n, int32_t dim, int32_t dtype,
                   void *dst, int64_t dst_pitch, float *scale)
{
    if (!src || !dst || n < 0 || dim <= 0)
        return -1;
    int esz = dtype == OR_F32 ? 4 : (dtype == OR_F16 || dtype == OR_BF16) ? 2 : 1;
    if (dst_pitch < (int64_t)dim * esz)
        return -1;
    if (dtype == OR_FP8 && !scale)
        return -1;
    for (int64_t i = 0; i < n; i++) {
        const float *x = src + i * dim;
        uint8_t *row = (uint8_t *)dst + i * dst_pitch;
        memset(row, 0, (size_t)dst_pitch);
        float s = 1.0f;
        if (dtype == OR_FP8) {
            float mx = 0.0f;
            for (int j = 0; j < dim; j++)
                if (fabsf(x[j]) > mx) mx = fabsf(x[j]);
            s = mx > 0.0f ? mx / 448.0f : 1.0f;
            scale[i] = s;
        }
        for (int j = 0; j < dim; j++) {
            if (dtype == OR_F32) {
                memcpy(row + 4 * j, &x[j], 4);
            } else if (dtype == OR_F16) {
                uint16_t c = (uint16_t)or_encode_f16(x[j]);
                memcpy(row + 2 * j, &c, 2);
            } else if (dtype == OR_BF16) {
                uint16_t c = (uint16_t)or_encode_bf16(x[j]);
                memcpy(row + 2 * j, &c, 2);
            } else if (dtype == OR_FP8) {
                float y = x[j] / s;
                row[j] = (uint8_t)or_encode_fp8(y);
            } else {
                return -1;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Distances                                                                  */
/* ------------------------------------------------------------------------- */

static double elem(const or_vecs *v, int64_t i, int32_t j)
{
    const uint8_t *row = (const uint8_t *)v->data + i * v->pitch;
    uint32_t code = 0;
    switch (v->dtype) {
    case OR_U8: code = row[j]; break;
    case OR_F32: memcpy(&code, row + 4 * j, 4); break;
    case OR_F16: case OR_BF16: { uint16_t c; memcpy(&c, row + 2 * j, 2); code = c; break; }
    case OR_FP8: code = row[j]; break;
    }
    double x = or_decode(v->dtype, code);
    if (v->dtype == OR_FP8)
        x *= (double)v->scale[i];
    return x;
}

double or_dist(const or_vecs *a, int64_t i, const or_vecs *b, int64_t j)
{
    if (a->dtype == OR_U8 && b->dtype == OR_U8 && a->metric == OR_L2SQ) {
        const uint8_t *x = (const uint8_t *)a->data + i * a->pitch;
        const uint8_t *y = (const uint8_t *)b->data + j * b->pitch;
        int64_t s = 0;
        for (int32_t t = 0; t < a->dim; t++) {
            int64_t diff = (int64_t)x[t] - (int64_t)y[t];
            s += diff * diff;
        }
        return (double)s;
    }
    double s = 0.0;
    if (a->metric == OR_L2SQ) {
        for (int32_t t = 0; t < a->dim; t++) {
            double diff = elem(a, i, t) - elem(b, j, t);
            s += diff * diff;
        }
        return s;
    }
    for (int32_t t = 0; t < a->dim; t++)
        s += elem(a, i, t) * elem(b, j, t);
    return 1.0 - s;
}

/* (d, id) total order */
static int key_less(double da, int64_t ia, double db, int64_t ib)
{
    return da < db || (da == db && ia < ib);
}

/* ------------------------------------------------------------------------- */
/* Exact top-k                                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_vecs *Q, *B;
    const int64_t *q_rows;
    const int32_t *cand;
    int64_t nq, ncand;
    int32_t k, exclude_self;
    int32_t *out_ids;
    double *out_d;
    int64_t next;
    pthread_mutex_t mu;
} topk_job;

static void topk_one(topk_job *J, int64_t r)
{
    int64_t qi = J->q_rows ? J->q_rows[r] : r;
    int32_t k = J->k;
    int32_t *ids = J->out_ids + r * k;
    double *ds = J->out_d + r * k;
    int32_t cnt = 0;
    for (int32_t t = 0; t < k; t++) { ids[t] = -1; ds[t] = INFINITY; }
    int64_t nc = J->cand ? J->ncand : J->B->n;
    for (int64_t c = 0; c < nc; c++) {
        int64_t j = J->cand ? J->cand[c] : c;
        if (J->exclude_self && j == qi)
            continue;
        double d = or_dist(J->Q, qi, J->B, j);
        /* keep the k smallest (d, j): sorted insertion into a bounded list */
        if (cnt == k && !key_less(d, j, ds[k - 1], ids[k - 1]))
            continue;
        int32_t pos = cnt < k ? cnt : k - 1;
        while (pos > 0 && key_less(d, j, ds[pos - 1], ids[pos - 1])) {
            ds[pos] = ds[pos - 1];
            ids[pos] = ids[pos - 1];
            pos--;
        }
        ds[pos] = d;
        ids[pos] = (int32_t)j;
        if (cnt < k) cnt++;
    }
}

static void *topk_worker(void *arg)
{
    topk_job *J = (topk_job *)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t r = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (r >= J->nq) break;
        topk_one(J, r);
    }
    return NULL;
}

static void run_pool(void *(*fn)(void *), void *arg, int32_t nthreads)
{
    if (nthreads <= 1) { fn(arg); return; }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int32_t t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, fn, arg);
    for (int32_t t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
}

int or_topk(const or_vecs *Q, const int64_t *q_rows, int64_t nq,
            const or_vecs *B, const int32_t *cand, int64_t ncand,
            int32_t k, int32_t exclude_self,
            int32_t *out_ids, double *out_d, int32_t nthreads)
{
    if (!Q || !B || k <= 0 || nq < 0 || !out_ids || !out_d || Q->dim != B->dim)
        return -1;
    topk_job J = {Q, B, q_rows, cand, nq, ncand, k, exclude_self, out_ids, out_d, 0,
                  PTHREAD_MUTEX_INITIALIZER};
    run_pool(topk_worker, &J, nthreads);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Edge set used by Algorithm 2: adjacency lists plus a (src,dst) hash set    */
/* ------------------------------------------------------------------------- */

typedef struct { int32_t *id; double *len; int32_t n, cap; } elist;

static void elist_push(elist *l, int32_t id, double len)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 8;
        l->id = (int32_t *)realloc(l->id, sizeof(int32_t) * (size_t)l->cap);
        l->len = (double *)realloc(l->len, sizeof(double) * (size_t)l->cap);
    }
    l->id[l->n] = id;
    l->len[l->n] = len;
    l->n++;
}

typedef struct { uint64_t *slot; uint64_t mask; } pairset;   /* 0 = empty */

static uint64_t mix64(uint64_t x)
{
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33; return x;
}

/* returns 1 if inserted, 0 if already present */
static int pairset_insert(pairset *s, int32_t a, int32_t b)
{
    uint64_t key = (((uint64_t)(uint32_t)a << 32) | (uint32_t)b) + 1;
    uint64_t h = mix64(key) & s->mask;
    while (s->slot[h]) {
        if (s->slot[h] == key) return 0;
        h = (h + 1) & s->mask;
    }
    s->slot[h] = key;
    return 1;
}

typedef struct { double len; int32_t id; } edge_t;

static int edge_cmp(const void *a, const void *b)
{
    const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
    if (x->len < y->len) return -1;
    if (x->len > y->len) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

static void sort_list(elist *l)
{
    edge_t *e = (edge_t *)malloc(sizeof(edge_t) * (size_t)(l->n ? l->n : 1));
    for (int32_t t = 0; t < l->n; t++) { e[t].len = l->len[t]; e[t].id = l->id[t]; }
    qsort(e, (size_t)l->n, sizeof(edge_t), edge_cmp);
    for (int32_t t = 0; t < l->n; t++) { l->len[t] = e[t].len; l->id[t] = e[t].id; }
    free(e);
}

static int64_t write_csr(elist *G, int64_t n, int64_t *off, int32_t *nbrs, double *lens,
                         int64_t cap)
{
    int64_t total = 0;
    for (int64_t o = 0; o < n; o++) total += G[o].n;
    if (!nbrs) return total;
    if (total > cap) return -total;
    int64_t p = 0;
    for (int64_t o = 0; o < n; o++) {
        off[o] = p;
        for (int32_t t = 0; t < G[o].n; t++) {
            nbrs[p] = G[o].id[t];
            lens[p] = G[o].len[t];
            p++;
        }
    }
    off[n] = p;
    return total;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 2: ConstructAdjustedGraph                                        */
/* ------------------------------------------------------------------------- */

int or_adjust_degree(const int32_t *knn_ids, const double *knn_d, int64_t n,
                     int32_t k, int32_t e_o, int32_t e_i,
                     int64_t *offsets, int32_t *nbrs, double *lens,
                     int64_t nnz_cap, int64_t *nnz_out)
{
    if (!knn_ids || !knn_d || n < 0 || k < 0 || e_o < 0 || e_i < 0 || !nnz_out)
        return -1;
    if (nbrs && (!offsets || !lens))
        return -1;
    elist *G = (elist *)calloc((size_t)(n ? n : 1), sizeof(elist));
    uint64_t cap = 1;
    while (cap < (uint64_t)(2 * n * (int64_t)(k ? k : 1) + 16)) cap <<= 1;
    pairset E = {(uint64_t *)calloc(cap, sizeof(uint64_t)), cap - 1};
    /* S <- N(G, o); the kNN row is S in ascending (d, id) order, so taking
     * argmin repeatedly is walking the row from the front. */
    char *taken = (char *)malloc((size_t)(k ? k : 1));
    for (int64_t o = 0; o < n; o++) {
        const int32_t *row = knn_ids + o * k;
        const double *rd = knn_d + o * k;
        int32_t rowlen = 0;
        while (rowlen < k && row[rowlen] >= 0) rowlen++;
        memset(taken, 0, (size_t)(k ? k : 1));
        int32_t remaining = rowlen;
        int32_t p = 1;
        while (remaining > 0 && (p <= e_o || p <= e_i)) {      /* R1 */
            int32_t best = -1;
            for (int32_t t = 0; t < rowlen; t++) {              /* argmin (d, id) */
                if (taken[t]) continue;
                if (best < 0 || key_less(rd[t], row[t], rd[best], row[best])) best = t;
            }
            taken[best] = 1;
            remaining--;
            int32_t nn = row[best];
            double len = rd[best];
            if (p <= e_o && pairset_insert(&E, (int32_t)o, nn))
                elist_push(&G[o], nn, len);
            if (p <= e_i && pairset_insert(&E, nn, (int32_t)o))
                elist_push(&G[nn], (int32_t)o, len);
            p++;
        }
    }
    free(taken);
    free(E.slot);
    for (int64_t o = 0; o < n; o++) sort_list(&G[o]);   /* edges sorted by length */
    int64_t total = write_csr(G, n, offsets, nbrs, lens, nnz_cap);
    for (int64_t o = 0; o < n; o++) { free(G[o].id); free(G[o].len); }
    free(G);
    *nnz_out = total < 0 ? -total : total;
    return total < 0 ? -3 : 0;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 3: ConstructAdjustedGraphWithConstraint                          */
/* ------------------------------------------------------------------------- */

static int elist_has(const elist *l, int32_t id)
{
    for (int32_t t = 0; t < l->n; t++)
        if (l->id[t] == id) return 1;
    return 0;
}

typedef struct { int64_t cnt, id; } mkey_t;

static int mkey_cmp(const void *a, const void *b)
{
    const mkey_t *x = (const mkey_t *)a, *y = (const mkey_t *)b;
    if (x->cnt != y->cnt) return x->cnt < y->cnt ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

int or_adjust_degree_constrained(const int32_t *knn_ids, const double *knn_d, int64_t n,
                                 int32_t k, int32_t e_o, int32_t e_i,
                                 int64_t *offsets, int32_t *nbrs, double *lens,
                                 int64_t nnz_cap, int64_t *nnz_out)
{
    if (!knn_ids || !knn_d || n < 0 || k < 0 || e_o < 0 || e_i < 0 || !nnz_out)
        return -1;
    if (nbrs && (!offsets || !lens))
        return -1;
    /* G_t <- ConstructAdjustedGraph(G, 0, e_i): the reverse edges only */
    int64_t tn = 0;
    if (or_adjust_degree(knn_ids, knn_d, n, k, 0, e_i, NULL, NULL, NULL, 0, &tn) != 0)
        return -1;
    int64_t *t_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *t_nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tn ? tn : 1));
    double *t_len = (double *)malloc(sizeof(double) * (size_t)(tn ? tn : 1));
    elist *Ge = (elist *)calloc((size_t)(n ? n : 1), sizeof(elist));
    /* G_i is kept only through its in-degrees: o joins N(G_i, n) at most once,
     * since o considers each member of N(G_t, o) once. */
    int64_t *indeg = (int64_t *)calloc((size_t)(n ? n : 1), sizeof(int64_t));
    mkey_t *M = (mkey_t *)malloc(sizeof(mkey_t) * (size_t)(n ? n : 1));
    int rc = or_adjust_degree(knn_ids, knn_d, n, k, 0, e_i, t_off, t_nb, t_len, tn, &tn);
    if (rc != 0) n = 0;
    /* M in the order the repeated argmin takes it: |N(G_t, x)| does not change
     * while M shrinks, so that order is ascending (|N(G_t, x)|, x) (R10). */
    for (int64_t x = 0; x < n; x++) { M[x].cnt = t_off[x + 1] - t_off[x]; M[x].id = x; }
    qsort(M, (size_t)n, sizeof(mkey_t), mkey_cmp);
    for (int64_t a = 0; a < n; a++) {
        int64_t o = M[a].id;
        /* S <- N(G_t, o).  Algorithm 2's lists come out in ascending (len, id)
         * order, so the repeated argmin over S walks the list from the front. */
        for (int64_t t = t_off[o]; t < t_off[o + 1]; t++) {
            int32_t nn = t_nb[t];
            if (indeg[nn] == 0 || (indeg[nn] < e_i && Ge[o].n < e_o)) {
                elist_push(&Ge[o], nn, t_len[t]);
                indeg[nn]++;
            }
        }
    }
    /* Fill every node up to e_o from its own k-NN row, which is S in ascending
     * (d, id) order; members already in N(G_e, o) are skipped. */
    for (int64_t o = 0; o < n; o++) {
        const int32_t *row = knn_ids + o * k;
        const double *rd = knn_d + o * k;
        for (int32_t t = 0; t < k && row[t] >= 0 && Ge[o].n < e_o; t++)
            if (!elist_has(&Ge[o], row[t]))
                elist_push(&Ge[o], row[t], rd[t]);
    }
    for (int64_t o = 0; o < n; o++) sort_list(&Ge[o]);   /* emitted in (len, id) order */
    int64_t total = write_csr(Ge, n, offsets, nbrs, lens, nnz_cap);
    for (int64_t o = 0; o < n; o++) { free(Ge[o].id); free(Ge[o].len); }
    free(Ge); free(indeg); free(M);
    free(t_off); free(t_nb); free(t_len);
    if (rc != 0) return -1;
    *nnz_out = total < 0 ? -total : total;
    return total < 0 ? -3 : 0;
}

/* ------------------------------------------------------------------------- */
/* Tree-based seeds: a 4-way vantage-point tree (Section 3.2, Table 5)        */
/* ------------------------------------------------------------------------- */

/* Distances inside the tree: exact integers on u8 (squared L2); on f32 rows
 * fp32 arithmetic in coordinate order, each product and sum rounded on its
 * own (squared L2, or 1 - dot for cosine).  These values decide branches,
 * so they are fixed to one precision and order (the tree is defined in it). */
static double vp_dist(const or_vecs *a, int64_t i, const or_vecs *b, int64_t j)
{
    if (a->dtype == OR_U8)
        return or_dist(a, i, b, j);
    const float *x = (const float *)((const uint8_t *)a->data + i * a->pitch);
    const float *y = (const float *)((const uint8_t *)b->data + j * b->pitch);
    float s = 0.0f;
    if (a->metric == OR_L2SQ) {
        for (int32_t t = 0; t < a->dim; t++) {
            float df = x[t] - y[t];
            float sq = df * df;
            s = s + sq;
        }
        return (double)s;
    }
    for (int32_t t = 0; t < a->dim; t++) {
        float pr = x[t] * y[t];
        s = s + pr;
    }
    return (double)(1.0f - s);
}

typedef struct { double d; int32_t id; } did_t;

static int did_cmp(const void *a, const void *b)
{
    const did_t *x = (const did_t *)a, *y = (const did_t *)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

static int32_t min_priority(const int32_t *ids, int64_t m, const uint32_t *prio)
{
    int32_t best = ids[0];
    for (int64_t t = 1; t < m; t++) {
        int32_t x = ids[t];
        if (prio[x] < prio[best] || (prio[x] == prio[best] && x < best)) best = x;
    }
    return best;
}

int or_vptree_build(const or_vecs *B, const uint32_t *prio, int32_t leaf_size, int32_t n_seeds,
                    int32_t *node_vp, int32_t *node_child, double *node_mu,
                    int32_t *leaf_seeds, int64_t *n_nodes, int64_t *n_leaves)
{
    int64_t n = B->n;
    if (n < 1 || leaf_size < 4 || n_seeds < 1) return -1;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *qb = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);   /* FIFO of segments */
    int64_t *qm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *qn = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    did_t *tmp = (did_t *)malloc(sizeof(did_t) * (size_t)n);
    for (int64_t t = 0; t < n; t++) perm[t] = (int32_t)t;
    int64_t head = 0, tail = 0, next = 1, leaves = 0;
    qb[tail] = 0; qm[tail] = n; qn[tail] = 0; tail++;
    while (head < tail) {                       /* breadth first: nodes numbered by level */
        int64_t b = qb[head], m = qm[head], node = qn[head];
        head++;
        int32_t *seg = perm + b;
        int32_t vp = min_priority(seg, m, prio);
        node_vp[node] = vp;
        if (m <= leaf_size) {
            /* leaf: its seeds are the n_seeds members nearest its vantage point */
            for (int64_t t = 0; t < m; t++) { tmp[t].id = seg[t]; tmp[t].d = vp_dist(B, vp, B, seg[t]); }
            qsort(tmp, (size_t)m, sizeof(did_t), did_cmp);
            for (int32_t r = 0; r < n_seeds; r++)
                leaf_seeds[leaves * n_seeds + r] = r < m ? tmp[r].id : -1;
            node_child[node] = (int32_t)(-1 - leaves);
            leaves++;
            continue;
        }
        /* the others in ascending (d(vp, x), x), cut into four runs of equal size */
        int64_t m1 = 0;
        for (int64_t t = 0; t < m; t++)
            if (seg[t] != vp) { tmp[m1].id = seg[t]; tmp[m1].d = vp_dist(B, vp, B, seg[t]); m1++; }
        qsort(tmp, (size_t)m1, sizeof(did_t), did_cmp);
        seg[0] = vp;
        for (int64_t t = 0; t < m1; t++) seg[1 + t] = tmp[t].id;
        node_child[node] = (int32_t)next;
        for (int32_t c = 0; c < 4; c++) {
            int64_t r0 = c * m1 / 4, r1 = (c + 1) * m1 / 4;
            if (c > 0) node_mu[3 * node + c - 1] = tmp[r0].d;
            qb[tail] = b + 1 + r0; qm[tail] = r1 - r0; qn[tail] = next + c; tail++;
        }
        next += 4;
    }
    *n_nodes = next;
    *n_leaves = leaves;
    free(perm); free(qb); free(qm); free(qn); free(tmp);
    return 0;
}

int or_vptree_seeds(const or_vecs *B, const or_vecs *Q, int64_t nq, const int32_t *node_vp,
                    const int32_t *node_child, const double *node_mu,
                    const int32_t *leaf_seeds, int32_t n_seeds, int32_t *seeds, int32_t *dc)
{
    for (int64_t q = 0; q < nq; q++) {
        int64_t node = 0;
        int32_t cnt = 0;
        while (node_child[node] >= 0) {
            double d = vp_dist(Q, q, B, node_vp[node]);
            cnt++;
            int c = (d >= node_mu[3 * node]) + (d >= node_mu[3 * node + 1]) +
                    (d >= node_mu[3 * node + 2]);
            node = node_child[node] + c;
        }
        int64_t leaf = -1 - (int64_t)node_child[node];
        for (int32_t r = 0; r < n_seeds; r++) seeds[q * n_seeds + r] = leaf_seeds[leaf * n_seeds + r];
        dc[q] = cnt;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Algorithms 4 and 5: AdjustPath / HasPath                                   */
/* ------------------------------------------------------------------------- */

/* HasPath(G_p, ns, nd): some n in N(G_p, ns) has nd in N(G_p, n) with
 * d(n, nd) < d(ns, nd).  Lists of G_p are in ascending (len, id) order
 * (edges are added in that order), so the scan of N(G_p, n) can stop at the
 * first length that is not smaller. */
static int has_path(const elist *Gp, int32_t ns, int32_t nd, double d_ns_nd)
{
    const elist *L = &Gp[ns];
    for (int32_t t = 0; t < L->n; t++) {
        const elist *M = &Gp[L->id[t]];
        for (int32_t u = 0; u < M->n && M->len[u] < d_ns_nd; u++)
            if (M->id[u] == nd)
                return 1;
    }
    return 0;
}

int or_adjust_path(const int64_t *in_off, const int32_t *in_nbrs,
                   const double *in_lens, int64_t n,
                   int64_t *out_off, int32_t *out_nbrs, double *out_lens,
                   int64_t *nnz_out)
{
    if (!in_off || n < 0 || !nnz_out)
        return -1;
    /* G_t: working copy, each list in ascending (len, id): its argmin is its
     * front, so removing the argmin advances a cursor. */
    elist *Gt = (elist *)calloc((size_t)(n ? n : 1), sizeof(elist));
    elist *Gp = (elist *)calloc((size_t)(n ? n : 1), sizeof(elist));
    int32_t *cur = (int32_t *)calloc((size_t)(n ? n : 1), sizeof(int32_t));
    for (int64_t v = 0; v < n; v++) {
        for (int64_t e = in_off[v]; e < in_off[v + 1]; e++)
            elist_push(&Gt[v], in_nbrs[e], in_lens[e]);
        sort_list(&Gt[v]);
    }
    /* V_t as an ascending list of nodes with remaining edges */
    int64_t *Vt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t nvt = 0;
    for (int64_t v = 0; v < n; v++)
        if (Gt[v].n > 0) Vt[nvt++] = v;
    while (nvt > 0) {
        int64_t keep = 0;
        for (int64_t t = 0; t < nvt; t++) {            /* FORALL n in V_t, ascending */
            int64_t v = Vt[t];
            int32_t nd = Gt[v].id[cur[v]];
            double len = Gt[v].len[cur[v]];
            if (!has_path(Gp, (int32_t)v, nd, len))
                elist_push(&Gp[v], nd, len);
            cur[v]++;                                   /* N(G_t,n) \ {n_d} */
            if (cur[v] < Gt[v].n)
                Vt[keep++] = v;                         /* else V_t \ {n} */
        }
        nvt = keep;
    }
    int64_t total = 0;
    for (int64_t v = 0; v < n; v++) total += Gp[v].n;
    if (out_nbrs) {
        if (!out_off || !out_lens) return -1;
        write_csr(Gp, n, out_off, out_nbrs, out_lens, total);
    }
    *nnz_out = total;
    for (int64_t v = 0; v < n; v++) {
        free(Gt[v].id); free(Gt[v].len); free(Gp[v].id); free(Gp[v].len);
    }
    free(Gt); free(Gp); free(cur); free(Vt);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Algorithms 6/7: visited-node table b plus collision lists L                */
/* ------------------------------------------------------------------------- */

int64_t or_hash_size(int64_t n, int32_t b)
{
    int32_t lg = 0;                         /* floor(log2 n), a bit operation */
    while (((int64_t)1 << (lg + 1)) <= n) lg++;
    return (int64_t)1 << ((lg + b) / 2);
}

typedef struct {
    int64_t s;
    int64_t *b;            /* first id per bucket, -1 = empty */
    int64_t *head;         /* collision list per bucket, -1 = empty */
    int64_t *lid, *lnext;  /* list node pool */
    int64_t nl, capl;
    int64_t *touched;      /* buckets to clear */
    int64_t ntouched;
} visited_t;

static void visited_init(visited_t *V, int64_t n)
{
    V->s = or_hash_size(n > 0 ? n : 1, 11);
    V->b = (int64_t *)malloc(sizeof(int64_t) * (size_t)V->s);
    V->head = (int64_t *)malloc(sizeof(int64_t) * (size_t)V->s);
    for (int64_t h = 0; h < V->s; h++) { V->b[h] = -1; V->head[h] = -1; }
    V->capl = 1024;
    V->lid = (int64_t *)malloc(sizeof(int64_t) * (size_t)V->capl);
    V->lnext = (int64_t *)malloc(sizeof(int64_t) * (size_t)V->capl);
    V->nl = 0;
    V->touched = (int64_t *)malloc(sizeof(int64_t) * (size_t)V->s);
    V->ntouched = 0;
}

static void visited_clear(visited_t *V)
{
    for (int64_t t = 0; t < V->ntouched; t++) {
        V->b[V->touched[t]] = -1;
        V->head[V->touched[t]] = -1;
    }
    V->ntouched = 0;
    V->nl = 0;
}

static void visited_free(visited_t *V)
{
    free(V->b); free(V->head); free(V->lid); free(V->lnext); free(V->touched);
}

static int visited_isset(const visited_t *V, int64_t i)     /* Algorithm 7 */
{
    int64_t h = i & (V->s - 1);             /* i mod s, s a power of two */
    if (V->b[h] == i) return 1;
    for (int64_t p = V->head[h]; p >= 0; p = V->lnext[p])
        if (V->lid[p] == i) return 1;
    return 0;
}

static void visited_set(visited_t *V, int64_t i)            /* Algorithm 6 */
{
    int64_t h = i & (V->s - 1);
    if (V->b[h] < 0) {
        V->b[h] = i;
        V->touched[V->ntouched++] = h;
    } else if (V->b[h] != i) {
        for (int64_t p = V->head[h]; p >= 0; p = V->lnext[p])
            if (V->lid[p] == i) return;     /* already in L_h */
        if (V->nl == V->capl) {
            V->capl *= 2;
            V->lid = (int64_t *)realloc(V->lid, sizeof(int64_t) * (size_t)V->capl);
            V->lnext = (int64_t *)realloc(V->lnext, sizeof(int64_t) * (size_t)V->capl);
        }
        V->lid[V->nl] = i;
        V->lnext[V->nl] = V->head[h];
        V->head[h] = V->nl++;
    }
}

int or_visited_replay(int64_t n, const int64_t *ops, int64_t nops, int32_t *answers)
{
    if (!ops || !answers || n <= 0) return -1;
    visited_t V;
    visited_init(&V, n);
    int64_t a = 0;
    for (int64_t t = 0; t < nops; t++) {
        if (ops[t] >= 0) visited_set(&V, ops[t]);
        else answers[a++] = visited_isset(&V, -ops[t] - 1);
    }
    visited_free(&V);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1: KnnSearch                                                     */
/* ------------------------------------------------------------------------- */

/* S: min-heap on (d, id) */
typedef struct { double d; int64_t id; } item_t;
typedef struct { item_t *a; int64_t n, cap; } heap_t;

static void heap_push(heap_t *h, double d, int64_t id)
{
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 64;
        h->a = (item_t *)realloc(h->a, sizeof(item_t) * (size_t)h->cap);
    }
    int64_t i = h->n++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!key_less(d, id, h->a[p].d, h->a[p].id)) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].d = d;
    h->a[i].id = id;
}

static item_t heap_pop(heap_t *h)
{
    item_t top = h->a[0];
    item_t last = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= h->n) break;
        if (c + 1 < h->n && key_less(h->a[c + 1].d, h->a[c + 1].id, h->a[c].d, h->a[c].id)) c++;
        if (!key_less(h->a[c].d, h->a[c].id, last.d, last.id)) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->n > 0) h->a[i] = last;
    return top;
}

/* R: the result set, kept as a list in ascending (d, id) */
typedef struct { double *d; int64_t *id; int32_t n, k; } rset_t;

/* Lines "if d <= r: R <- R u {n}; if |R| > k remove argmax; if |R| = k r <- max". */
static void rset_offer(rset_t *R, double *r, double d, int64_t id)
{
    if (!(d <= *r)) return;
    int32_t pos = R->n;
    while (pos > 0 && key_less(d, id, R->d[pos - 1], R->id[pos - 1])) {
        R->d[pos] = R->d[pos - 1];
        R->id[pos] = R->id[pos - 1];
        pos--;
    }
    R->d[pos] = d;
    R->id[pos] = id;
    R->n++;
    if (R->n > R->k) R->n--;                /* drop argmax (d, id): the last */
    if (R->n == R->k) *r = R->d[R->n - 1];
}

typedef struct {
    const or_vecs *base, *queries;
    const int64_t *off;
    const int32_t *nbrs;
    int64_t n_nodes, nq;
    const int32_t *seeds;
    int32_t n_seeds;
    const int32_t *k;
    const float *eps, *eps1;
    const uint32_t *ep, *ep1;
    int32_t probe_hops;
    const int32_t *max_dc;
    int32_t k_stride;
    int32_t *out_ids;
    double *out_d;
    int64_t *out_dc, *out_hops;
    double *out_margin, *feat;
    int32_t pool_k;
    int32_t *pool_ids;
    double *pool_d, *pool_margin;
    int32_t probe_only;
    int64_t next;
    pthread_mutex_t mu;
} search_job;

/* The candidates of a rerank: the pool_k + 1 smallest (d, id) among the
 * distances the search computed (seeds and visited nodes), ascending. */
typedef struct { double *d; int64_t *id; int32_t n, cap; } pool_t;

static void pool_offer(pool_t *P, double d, int64_t id)
{
    if (P->cap == 0) return;
    if (P->n == P->cap && !key_less(d, id, P->d[P->n - 1], P->id[P->n - 1])) return;
    int32_t pos = P->n < P->cap ? P->n : P->cap - 1;
    while (pos > 0 && key_less(d, id, P->d[pos - 1], P->id[pos - 1])) {
        P->d[pos] = P->d[pos - 1];
        P->id[pos] = P->id[pos - 1];
        pos--;
    }
    P->d[pos] = d;
    P->id[pos] = id;
    if (P->n < P->cap) P->n++;
}

/* f of reading R5 */
static float range_factor(float eps, int32_t metric)
{
    if (isinf(eps)) return INFINITY;
    double t = 1.0 + (double)eps;
    return metric == OR_L2SQ ? (float)(t * t) : (float)t;
}

/* thr(r) of reading R5 */
static double threshold(double r, float f, int u8)
{
    if (isinf(r) || isinf(f)) return INFINITY;
    if (u8) {
        volatile float rf = (float)r;
        volatile float t = rf * f;          /* one fp32 multiply */
        return (double)t;
    }
    return r * (double)f;
}

static double rel_gap(double a, double b, double floor_)
{
    if (isinf(a) || isinf(b)) return INFINITY;
    double m = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
    if (m < floor_) m = floor_;
    return fabs(a - b) / m;
}

static int dcmp(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

static void search_one(search_job *J, visited_t *C, heap_t *S, rset_t *R, pool_t *Pl, int64_t q)
{
    const int u8 = J->base->dtype == OR_U8;
    const double mfloor = J->base->metric == OR_COS ? 1e-2 : 1e-300;
    const int32_t k = J->k[q];
    double margin = INFINITY;
    int64_t dc = 0, hops = 0;
    double r = INFINITY;
    float f = range_factor(J->eps[q], J->base->metric);
    uint32_t ep = J->ep[q];
    int phase1 = J->eps1 != NULL;
    if (phase1) {
        f = range_factor(J->eps1[q], J->base->metric);
        ep = J->ep1[q];
    }
    visited_clear(C);
    S->n = 0;
    R->n = 0;
    R->k = k;
    Pl->n = 0;
    double seedd[64];
    int32_t nseedd = 0;

    /* S <- Seed(G), R from the seeds (R2) */
    for (int32_t t = 0; t < J->n_seeds; t++) {
        int64_t s = J->seeds[q * J->n_seeds + t];
        if (s < 0 || s >= J->n_nodes || visited_isset(C, s)) continue;
        visited_set(C, s);
        double d = or_dist(J->base, s, J->queries, q);
        dc++;
        if (nseedd < 64) seedd[nseedd++] = d;
        if (!isinf(r)) margin = fmin(margin, rel_gap(d, r, mfloor));
        rset_offer(R, &r, d, s);
        pool_offer(Pl, d, s);
        heap_push(S, d, s);
    }
    const int64_t budget = J->max_dc && J->max_dc[q] > 0 ? J->max_dc[q] : INT64_MAX;
    while (S->n > 0) {
        if (dc >= budget) break;                            /* budget spent */
        item_t s = heap_pop(S);
        double thr = threshold(r, f, u8);
        if (S->n > 0) margin = fmin(margin, rel_gap(s.d, S->a[0].d, mfloor));
        margin = fmin(margin, rel_gap(s.d, thr, mfloor));
        if (s.d > thr) break;                               /* d(s,q) > r(1+eps) */
        hops++;
        uint32_t p = 1;
        for (int64_t e = J->off[s.id]; e < J->off[s.id + 1] && p <= ep; e++, p++) {
            int64_t nn = J->nbrs[e];                        /* argmin d(x, s): stored order */
            if (visited_isset(C, nn)) continue;
            visited_set(C, nn);
            double d = or_dist(J->base, nn, J->queries, q);
            dc++;
            thr = threshold(r, f, u8);
            margin = fmin(margin, rel_gap(d, thr, mfloor));
            if (d <= thr) heap_push(S, d, nn);
            margin = fmin(margin, rel_gap(d, r, mfloor));
            rset_offer(R, &r, d, nn);
            pool_offer(Pl, d, nn);
        }
        if (phase1 && hops == J->probe_hops) {
            if (J->feat) {
                double *F = J->feat + q * OR_NFEAT;
                qsort(seedd, (size_t)nseedd, sizeof(double), dcmp);
                for (int32_t t = 0; t < 8; t++)
                    F[t] = nseedd == 0 ? 0.0 : seedd[t < nseedd ? t : nseedd - 1];
                double rmax = R->n > 0 ? R->d[R->n - 1] : 0.0;
                F[8] = (double)S->n;
                if (S->n > 0) {
                    /* statistics of the m = min(|S|, 64) smallest entries of S */
                    double *tmp = (double *)malloc(sizeof(double) * (size_t)S->n);
                    for (int64_t t = 0; t < S->n; t++) tmp[t] = S->a[t].d;
                    qsort(tmp, (size_t)S->n, sizeof(double), dcmp);
                    int64_t m = S->n < 64 ? S->n : 64;
                    F[9] = tmp[0];
                    F[10] = tmp[(m + 1) / 2 - 1];
                    F[11] = tmp[m - 1];
                    free(tmp);
                } else {
                    F[9] = F[10] = F[11] = rmax;
                }
                F[12] = rmax;
                F[13] = (double)dc;
            }
            if (J->probe_only) break;   /* the state at the switch is all this call reports */
            f = range_factor(J->eps[q], J->base->metric);
            ep = J->ep[q];
        }
    }
    /* R ordered by (d, id); the k-th vs (k+1)-th margin is covered by the
     * R-insertion tests above. */
    int32_t *ids = J->out_ids + q * J->k_stride;
    double *ds = J->out_d + q * J->k_stride;
    for (int32_t t = 0; t < J->k_stride; t++) {
        ids[t] = t < R->n ? (int32_t)R->id[t] : -1;
        ds[t] = t < R->n ? R->d[t] : INFINITY;
    }
    if (J->out_dc) J->out_dc[q] = dc;
    if (J->out_hops) J->out_hops[q] = hops;
    if (J->out_margin) J->out_margin[q] = margin;
    if (J->pool_k > 0) {
        int32_t *pid = J->pool_ids + q * J->pool_k;
        double *pd = J->pool_d + q * J->pool_k;
        for (int32_t t = 0; t < J->pool_k; t++) {
            pid[t] = t < Pl->n ? (int32_t)Pl->id[t] : -1;
            pd[t] = t < Pl->n ? Pl->d[t] : INFINITY;
        }
        /* membership of the pool_k-th against the next distance computed */
        if (J->pool_margin)
            J->pool_margin[q] = Pl->n > J->pool_k
                ? rel_gap(Pl->d[J->pool_k - 1], Pl->d[J->pool_k], mfloor) : INFINITY;
    }
}

static void *search_worker(void *arg)
{
    search_job *J = (search_job *)arg;
    visited_t C;
    visited_init(&C, J->n_nodes);
    heap_t S = {NULL, 0, 0};
    int32_t kmax = 1;
    for (int64_t q = 0; q < J->nq; q++) if (J->k[q] > kmax) kmax = J->k[q];
    rset_t R;
    R.d = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    R.id = (int64_t *)malloc(sizeof(int64_t) * (size_t)(kmax + 1));
    pool_t Pl;
    Pl.cap = J->pool_k > 0 ? J->pool_k + 1 : 0;
    Pl.n = 0;
    Pl.d = (double *)malloc(sizeof(double) * (size_t)(Pl.cap + 1));
    Pl.id = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Pl.cap + 1));
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t q = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (q >= J->nq) break;
        search_one(J, &C, &S, &R, &Pl, q);
    }
    visited_free(&C);
    free(S.a); free(R.d); free(R.id); free(Pl.d); free(Pl.id);
    return NULL;
}

int or_search(const or_vecs *base, const int64_t *offsets, const int32_t *nbrs,
              int64_t n_nodes, const or_vecs *queries, int64_t nq,
              const int32_t *seeds, int32_t n_seeds,
              const int32_t *k, const float *eps, const uint32_t *ep,
              const float *eps1, const uint32_t *ep1, int32_t probe_hops,
              const int32_t *max_dc, int32_t k_stride, int32_t *out_ids, double *out_d,
              int64_t *out_dc, int64_t *out_hops, double *out_margin,
              double *feat, int32_t pool_k, int32_t *pool_ids, double *pool_d,
              double *pool_margin, int32_t probe_only, int32_t nthreads)
{
    if (!base || !offsets || !queries || !seeds || !k || !eps || !ep || !out_ids || !out_d)
        return -1;
    if (pool_k < 0 || (pool_k > 0 && (!pool_ids || !pool_d)))
        return -1;
    if (n_nodes != base->n || base->dim != queries->dim || n_seeds <= 0 || k_stride <= 0)
        return -1;
    if ((eps1 == NULL) != (ep1 == NULL) || (probe_only && !eps1))
        return -1;
    for (int64_t q = 0; q < nq; q++)
        if (k[q] <= 0 || k[q] > k_stride) return -1;
    search_job J = {base, queries, offsets, nbrs, n_nodes, nq, seeds, n_seeds, k, eps, eps1,
                    ep, ep1, probe_hops < 1 ? 1 : probe_hops, max_dc, k_stride, out_ids, out_d, out_dc,
                    out_hops, out_margin, feat, pool_k, pool_ids, pool_d, pool_margin,
                    probe_only, 0, PTHREAD_MUTEX_INITIALIZER};
    run_pool(search_worker, &J, nthreads);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Exact rerank of a candidate pool                                           */
/* ------------------------------------------------------------------------- */

int or_rerank(const or_vecs *Q, const or_vecs *B, const int32_t *pool, int32_t pool_sz,
              int64_t nq, int32_t k, int32_t *out_ids, double *out_d)
{
    if (!Q || !B || !pool || pool_sz < 0 || k <= 0 || !out_ids || !out_d)
        return -1;
    for (int64_t q = 0; q < nq; q++) {
        int32_t *ids = out_ids + q * k;
        double *ds = out_d + q * k;
        int32_t cnt = 0;
        for (int32_t t = 0; t < k; t++) { ids[t] = -1; ds[t] = INFINITY; }
        for (int32_t c = 0; c < pool_sz; c++) {
            int32_t j = pool[q * pool_sz + c];
            if (j < 0) continue;
            double d = or_dist(Q, q, B, j);
            if (cnt == k && !key_less(d, j, ds[k - 1], ids[k - 1])) continue;
            int32_t pos = cnt < k ? cnt : k - 1;
            while (pos > 0 && key_less(d, j, ds[pos - 1], ids[pos - 1])) {
                ds[pos] = ds[pos - 1];
                ids[pos] = ids[pos - 1];
                pos--;
            }
            ds[pos] = d;
            ids[pos] = j;
            if (cnt < k) cnt++;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* 2-layer MLP, fp64                                                          */
/* ------------------------------------------------------------------------- */

int or_mlp_forward(const double *X, int32_t batch, int32_t F,
                   const double *W1, const double *b1, int32_t H,
                   const double *W2, const double *b2, int32_t T,
                   double *hidden, double *Y)
{
    if (!X || !W1 || !b1 || !W2 || !b2 || !Y || batch < 0 || F <= 0 || H <= 0 || T <= 0)
        return -1;
    double *h = (double *)malloc(sizeof(double) * (size_t)H);
    for (int32_t n = 0; n < batch; n++) {
        for (int32_t j = 0; j < H; j++) {
            double a = b1[j];
            for (int32_t i = 0; i < F; i++) a += W1[j * F + i] * X[n * F + i];
            h[j] = a > 0.0 ? a : 0.0;                       /* ReLU */
            if (hidden) hidden[n * H + j] = h[j];
        }
        for (int32_t t = 0; t < T; t++) {
            double y = b2[t];
            for (int32_t j = 0; j < H; j++) y += W2[t * H + j] * h[j];
            Y[n * T + t] = y;
        }
    }
    free(h);
    return 0;
}

double or_mlp_loss_grad(const double *X, const double *target, const double *w,
                        int32_t batch, int32_t F,
                        const double *W1, const double *b1, int32_t H,
                        const double *W2, const double *b2, int32_t T,
                        double *gW1, double *gb1, double *gW2, double *gb2)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)H);
    double *h = (double *)malloc(sizeof(double) * (size_t)H);
    double *dy = (double *)malloc(sizeof(double) * (size_t)T);
    double *dh = (double *)malloc(sizeof(double) * (size_t)H);
    memset(gW1, 0, sizeof(double) * (size_t)H * (size_t)F);
    memset(gb1, 0, sizeof(double) * (size_t)H);
    memset(gW2, 0, sizeof(double) * (size_t)T * (size_t)H);
    memset(gb2, 0, sizeof(double) * (size_t)T);
    const double scale = 1.0 / ((double)batch * (double)T);
    double loss = 0.0;
    for (int32_t n = 0; n < batch; n++) {
        for (int32_t j = 0; j < H; j++) {
            double s = b1[j];
            for (int32_t i = 0; i < F; i++) s += W1[j * F + i] * X[n * F + i];
            a[j] = s;
            h[j] = s > 0.0 ? s : 0.0;
        }
        for (int32_t t = 0; t < T; t++) {
            double y = b2[t];
            for (int32_t j = 0; j < H; j++) y += W2[t * H + j] * h[j];
            double wt = w ? w[n * T + t] : 1.0;
            double e = y - target[n * T + t];
            loss += wt * e * e;
            dy[t] = 2.0 * wt * e * scale;                   /* dL/dy */
        }
        for (int32_t j = 0; j < H; j++) {
            double s = 0.0;
            for (int32_t t = 0; t < T; t++) s += W2[t * H + j] * dy[t];
            dh[j] = a[j] > 0.0 ? s : 0.0;                   /* through ReLU */
        }
        for (int32_t t = 0; t < T; t++) {
            gb2[t] += dy[t];
            for (int32_t j = 0; j < H; j++) gW2[t * H + j] += dy[t] * h[j];
        }
        for (int32_t j = 0; j < H; j++) {
            gb1[j] += dh[j];
            for (int32_t i = 0; i < F; i++) gW1[j * F + i] += dh[j] * X[n * F + i];
        }
    }
    free(a); free(h); free(dy); free(dh);
    return loss * scale;
}

void or_adam_step(double *p, const double *g, double *m, double *v, int64_t n,
                  double lr, double beta1, double beta2, double eps, int32_t t)
{
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; i++) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
