/*
 * Plain single-threaded CPU oracle for the three-way joins.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * What it computes is the plain relational definition (Sec. 3 and Sec. 5 of
 * the paper: R(AB) join S(BC) join T(CD), resp. T(CA); bags, no duplicate
 * elimination, Example 1's footnote; the result is aggregated by COUNT rather
 * than materialised, Sec. 6).  Every loop below is a nested-loop join whose
 * inner loops are restricted, through a sorted copy and binary search, to
 * the tuples that satisfy the join predicate.  Sorting and searching only
 * select tuples; they change no count.
 *
 * Keys are 32-bit patterns compared for equality.  Sums are carried in
 * unsigned 128-bit integers; a result that does not fit 64 bits is flagged.
 *
 * Relations are passed as two column pointers and an element stride
 * (stride 2 with col1 == col0 + 1 is a row-major [n, 2] array).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { ORC_OK = 0, ORC_OVERFLOW = 1, ORC_KEY_RANGE = 2, ORC_NOMEM = 3 };

/* ------------------------------------------------------------------------ */
/* small helpers: pairs (key, val) sorted by key then val                    */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t key, val; } pair_t;

static int cmp_pair(const void* x, const void* y) {
    const pair_t* p = (const pair_t*)x;
    const pair_t* q = (const pair_t*)y;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    if (p->val != q->val) return p->val < q->val ? -1 : 1;
    return 0;
}

static int cmp_u32(const void* x, const void* y) {
    uint32_t p = *(const uint32_t*)x, q = *(const uint32_t*)y;
    return p < q ? -1 : (p > q ? 1 : 0);
}

/* copy a relation into pairs with key = column kcol, val = the other one */
static pair_t* load_pairs(const uint32_t* c0, const uint32_t* c1, int64_t stride,
                          uint64_t n, int kcol) {
    pair_t* p = (pair_t*)malloc((n ? n : 1) * sizeof(pair_t));
    if (!p) return NULL;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t x = c0[i * stride], y = c1[i * stride];
        p[i].key = kcol == 0 ? x : y;
        p[i].val = kcol == 0 ? y : x;
    }
    qsort(p, n, sizeof(pair_t), cmp_pair);
    return p;
}

/* first index in p[lo, hi) whose key is >= k */
static uint64_t lower_key(const pair_t* p, uint64_t lo, uint64_t hi, uint32_t k) {
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (p[mid].key < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}
/* first index in p[lo, hi) whose key is > k */
static uint64_t upper_key(const pair_t* p, uint64_t lo, uint64_t hi, uint32_t k) {
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (p[mid].key <= k) lo = mid + 1; else hi = mid;
    }
    return lo;
}
/* first index in p[lo, hi) (all with one key, vals sorted) with val >= v */
static uint64_t lower_val(const pair_t* p, uint64_t lo, uint64_t hi, uint32_t v) {
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (p[mid].val < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
static uint64_t upper_val(const pair_t* p, uint64_t lo, uint64_t hi, uint32_t v) {
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (p[mid].val <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
static uint64_t lower_u32(const uint32_t* a, uint64_t n, uint32_t k) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}
static uint64_t upper_u32(const uint32_t* a, uint64_t n, uint32_t k) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] <= k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* Linear join, per-A count (Sec. 3 problem statement, Example 1's query).   */
/*   out[a] = #{ (r, s, t) : r.a = a, r.b = s.b, s.c = t.c }                 */
/* T's D column never takes part in a predicate, so for each s the inner     */
/* loop over t contributes the number of t with t.c = s.c.                   */
/* Returns ORC_KEY_RANGE if some r.a >= a_domain (out untouched), else       */
/* ORC_OVERFLOW if some out[a] needs more than 64 bits, else ORC_OK.         */
/* ------------------------------------------------------------------------ */
int orc_linear3_count(const uint32_t* r0, const uint32_t* r1, int64_t rstride, uint64_t nr,
                      const uint32_t* s0, const uint32_t* s1, int64_t sstride, uint64_t ns,
                      const uint32_t* t0, int64_t tstride, uint64_t nt,
                      uint32_t a_domain, uint64_t* out) {
    for (uint64_t i = 0; i < nr; ++i)
        if (r0[i * rstride] >= a_domain) return ORC_KEY_RANGE;

    /* T's C column, sorted */
    uint32_t* tc = (uint32_t*)malloc((nt ? nt : 1) * sizeof(uint32_t));
    /* S as (b, c) sorted by b */
    pair_t* s = load_pairs(s0, s1, sstride, ns, 0);
    u128* acc = (u128*)calloc(a_domain ? a_domain : 1, sizeof(u128));
    if (!tc || !s || !acc) { free(tc); free(s); free(acc); return ORC_NOMEM; }
    for (uint64_t i = 0; i < nt; ++i) tc[i] = t0[i * tstride];
    qsort(tc, nt, sizeof(uint32_t), cmp_u32);

    for (uint64_t i = 0; i < nr; ++i) {
        uint32_t a = r0[i * rstride], b = r1[i * rstride];
        uint64_t lo = lower_key(s, 0, ns, b), hi = upper_key(s, lo, ns, b);
        for (uint64_t j = lo; j < hi; ++j) {            /* s with s.b = r.b */
            uint32_t c = s[j].val;
            uint64_t nmatch = upper_u32(tc, nt, c) - lower_u32(tc, nt, c);  /* t with t.c = s.c */
            acc[a] += nmatch;
        }
    }
    int status = ORC_OK;
    for (uint32_t a = 0; a < a_domain; ++a) {
        if (acc[a] >> 64) status = ORC_OVERFLOW;
        out[a] = (uint64_t)acc[a];
    }
    free(tc); free(s); free(acc);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Size of the binary intermediate R(AB) join S(BC) on B (Sec. 6.3, the      */
/* first join of the cascade): #{ (r, s) : r.b = s.b }.                      */
/* ------------------------------------------------------------------------ */
int orc_join2_size(const uint32_t* r0, const uint32_t* r1, int64_t rstride, uint64_t nr,
                   const uint32_t* s0, int64_t sstride, uint64_t ns, uint64_t* out) {
    (void)r0;
    uint32_t* sb = (uint32_t*)malloc((ns ? ns : 1) * sizeof(uint32_t));
    if (!sb) return ORC_NOMEM;
    for (uint64_t i = 0; i < ns; ++i) sb[i] = s0[i * sstride];
    qsort(sb, ns, sizeof(uint32_t), cmp_u32);
    u128 total = 0;
    for (uint64_t i = 0; i < nr; ++i) {
        uint32_t b = r1[i * rstride];
        total += upper_u32(sb, ns, b) - lower_u32(sb, ns, b);
    }
    free(sb);
    *out = (uint64_t)total;
    return (total >> 64) ? ORC_OVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cyclic join R(AB) join S(BC) join T(CA), total count (Sec. 5).            */
/*   total = #{ (r, s, t) : r.b = s.b, s.c = t.c, t.a = r.a }                */
/* For each s the pairs (r, t) it joins with are those whose A values are    */
/* equal, with r from R's tuples of B = s.b and t from T's tuples of         */
/* C = s.c; the loop walks the shorter of the two lists and counts, for      */
/* each of its tuples, the tuples of the other list with the same A.         */
/* ------------------------------------------------------------------------ */
int orc_triangle3_count(const uint32_t* r0, const uint32_t* r1, int64_t rstride, uint64_t nr,
                        const uint32_t* s0, const uint32_t* s1, int64_t sstride, uint64_t ns,
                        const uint32_t* t0, const uint32_t* t1, int64_t tstride, uint64_t nt,
                        uint64_t* out_lo, uint64_t* out_hi) {
    pair_t* R = load_pairs(r0, r1, rstride, nr, 1);   /* key b, val a */
    pair_t* T = load_pairs(t0, t1, tstride, nt, 0);   /* key c, val a */
    if (!R || !T) { free(R); free(T); return ORC_NOMEM; }
    u128 total = 0;
    for (uint64_t i = 0; i < ns; ++i) {
        uint32_t b = s0[i * sstride], c = s1[i * sstride];
        uint64_t rlo = lower_key(R, 0, nr, b), rhi = upper_key(R, rlo, nr, b);
        uint64_t tlo = lower_key(T, 0, nt, c), thi = upper_key(T, tlo, nt, c);
        const pair_t* short_list = R; uint64_t slo = rlo, shi = rhi;
        const pair_t* long_list = T;  uint64_t llo = tlo, lhi = thi;
        if (rhi - rlo > thi - tlo) {
            short_list = T; slo = tlo; shi = thi;
            long_list = R;  llo = rlo; lhi = rhi;
        }
        for (uint64_t j = slo; j < shi; ++j) {
            uint32_t a = short_list[j].val;
            uint64_t lo = lower_val(long_list, llo, lhi, a);
            uint64_t hi = upper_val(long_list, lo, lhi, a);
            total += hi - lo;
        }
    }
    free(R); free(T);
    *out_lo = (uint64_t)total;
    *out_hi = (uint64_t)(total >> 64);
    return (total >> 64) ? ORC_OVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cyclic join restricted to a subset of S given by a 0/1 mask: used to      */
/* check a large join on a sample of S (the total is a sum over S tuples).   */
/* ------------------------------------------------------------------------ */
int orc_triangle3_count_masked(const uint32_t* r0, const uint32_t* r1, int64_t rstride, uint64_t nr,
                               const uint32_t* s0, const uint32_t* s1, int64_t sstride, uint64_t ns,
                               const uint8_t* smask,
                               const uint32_t* t0, const uint32_t* t1, int64_t tstride, uint64_t nt,
                               uint64_t* out_lo, uint64_t* out_hi) {
    uint64_t m = 0;
    for (uint64_t i = 0; i < ns; ++i) m += smask[i] != 0;
    uint32_t* sb = (uint32_t*)malloc((m ? m : 1) * 2 * sizeof(uint32_t));
    if (!sb) return ORC_NOMEM;
    uint64_t k = 0;
    for (uint64_t i = 0; i < ns; ++i)
        if (smask[i]) { sb[2 * k] = s0[i * sstride]; sb[2 * k + 1] = s1[i * sstride]; ++k; }
    int st = orc_triangle3_count(r0, r1, rstride, nr, sb, sb + 1, 2, m, t0, t1, tstride, nt,
                                 out_lo, out_hi);
    free(sb);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Linear join restricted to the R tuples whose A value is in a sorted list  */
/* of sampled A values: out[i] = count for a = alist[i].  Used to check the  */
/* full-size per-A counts on a sample of A values.                           */
/* ------------------------------------------------------------------------ */
int orc_linear3_count_sampled(const uint32_t* r0, const uint32_t* r1, int64_t rstride, uint64_t nr,
                              const uint32_t* s0, const uint32_t* s1, int64_t sstride, uint64_t ns,
                              const uint32_t* t0, int64_t tstride, uint64_t nt,
                              const uint32_t* alist, uint64_t na, uint64_t* out) {
    uint32_t* tc = (uint32_t*)malloc((nt ? nt : 1) * sizeof(uint32_t));
    pair_t* s = load_pairs(s0, s1, sstride, ns, 0);
    u128* acc = (u128*)calloc(na ? na : 1, sizeof(u128));
    if (!tc || !s || !acc) { free(tc); free(s); free(acc); return ORC_NOMEM; }
    for (uint64_t i = 0; i < nt; ++i) tc[i] = t0[i * tstride];
    qsort(tc, nt, sizeof(uint32_t), cmp_u32);
    for (uint64_t i = 0; i < nr; ++i) {
        uint32_t a = r0[i * rstride], b = r1[i * rstride];
        uint64_t ia = lower_u32(alist, na, a);
        if (ia == na || alist[ia] != a) continue;
        uint64_t lo = lower_key(s, 0, ns, b), hi = upper_key(s, lo, ns, b);
        for (uint64_t j = lo; j < hi; ++j) {
            uint32_t c = s[j].val;
            acc[ia] += upper_u32(tc, nt, c) - lower_u32(tc, nt, c);
        }
    }
    int status = ORC_OK;
    for (uint64_t i = 0; i < na; ++i) {
        if (acc[i] >> 64) status = ORC_OVERFLOW;
        out[i] = (uint64_t)acc[i];
    }
    free(tc); free(s); free(acc);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Distinct count of the linear join's D values per A, estimated with a     */
/* Flajolet-Martin sketch (the footnotes to Example 1 and to Sec. 4's step  */
/* list: the union of overlapping sets of friends of friends of friends,    */
/* each kept as a small sketch).  For each requested a the exact set        */
/*   D(a) = { t.d : r.a = a, r.b = s.b, s.c = t.c }                          */
/* is collected (level by level, below), its size reported, and its sketch  */
/* built element by element:                                                 */
/*   h = MurmurHash3's 32-bit finaliser of (d xor seed);                     */
/*   bitmap j = the low 4 bits of h (16 bitmaps of 32 bits, stochastic       */
/*   averaging); bit r = the number of trailing zeros of h >> 4 (28 when     */
/*   h >> 4 is zero).                                                        */
/* The estimate is Flajolet and Martin's: with R_j the lowest zero bit of    */
/* bitmap j, E = (16 / 0.77351) * 2^(sum R_j / 16), and 0 for an empty set.  */
/* ------------------------------------------------------------------------ */
static uint32_t fm_mix(uint32_t x, uint32_t seed) {
    uint32_t h = x ^ seed;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

static uint32_t ctz32(uint32_t x) {           /* x != 0 */
    uint32_t n = 0;
    while (!(x & 1u)) { x >>= 1; ++n; }
    return n;
}

static void fm_add(uint32_t* sk, uint32_t d, uint32_t seed) {
    uint32_t h = fm_mix(d, seed);
    uint32_t rest = h >> 4;
    sk[h & 15u] |= 1u << (rest ? ctz32(rest) : 28u);
}

static double fm_estimate(const uint32_t* sk) {
    int any = 0;
    uint32_t sum = 0;
    for (int j = 0; j < 16; ++j) {
        if (sk[j]) any = 1;
        sum += sk[j] == 0xFFFFFFFFu ? 32u : ctz32(~sk[j]);
    }
    if (!any) return 0.0;
    /* 2^(sum / 16) as a product of exact powers of two and 2^(1/16)^k */
    double p = 1.0;
    for (uint32_t i = 0; i < sum / 16; ++i) p *= 2.0;
    double f = 1.0;
    for (uint32_t i = 0; i < sum % 16; ++i) f *= 1.0442737824274138;   /* 2^(1/16) */
    return 16.0 / 0.77351 * p * f;
}

/* grow *buf (capacity *cap) to hold at least need values */
static int reserve_u32(uint32_t** buf, uint64_t* cap, uint64_t need) {
    if (need <= *cap) return 1;
    uint64_t c = *cap ? *cap : 1024;
    while (c < need) c *= 2;
    uint32_t* g = (uint32_t*)realloc(*buf, c * sizeof(uint32_t));
    if (!g) return 0;
    *buf = g;
    *cap = c;
    return 1;
}

/* sort and drop repeats; returns the new length */
static uint64_t sort_unique(uint32_t* v, uint64_t n) {
    qsort(v, n, sizeof(uint32_t), cmp_u32);
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; ++i)
        if (m == 0 || v[i] != v[m - 1]) v[m++] = v[i];
    return m;
}

/* D(a) level by level: B(a) = { r.b : r.a = a }, C(a) = { s.c : s.b in
 * B(a) }, D(a) = { t.d : t.c in C(a) } -- the same set as the paths
 * (a, b, c, d) give, without enumerating the paths. */
int orc_linear3_distinct(const uint32_t* r0, const uint32_t* r1, int64_t rstride, uint64_t nr,
                         const uint32_t* s0, const uint32_t* s1, int64_t sstride, uint64_t ns,
                         const uint32_t* t0, const uint32_t* t1, int64_t tstride, uint64_t nt,
                         const uint32_t* alist, uint64_t na, uint32_t seed,
                         uint32_t* sketch, double* est, uint64_t* exact) {
    pair_t* r = load_pairs(r0, r1, rstride, nr, 0);   /* (a, b) by a */
    pair_t* s = load_pairs(s0, s1, sstride, ns, 0);   /* (b, c) by b */
    pair_t* t = load_pairs(t0, t1, tstride, nt, 0);   /* (c, d) by c */
    uint32_t *bs = NULL, *cs = NULL, *ds = NULL;
    uint64_t bcap = 0, ccap = 0, dcap = 0;
    int status = ORC_OK;
    if (!r || !s || !t) { status = ORC_NOMEM; goto done; }
    for (uint64_t q = 0; q < na; ++q) {
        const uint32_t a = alist[q];
        uint64_t rlo = lower_key(r, 0, nr, a), rhi = upper_key(r, rlo, nr, a);
        uint64_t nb = 0, nc = 0, nd = 0;
        if (!reserve_u32(&bs, &bcap, rhi - rlo)) { status = ORC_NOMEM; goto done; }
        for (uint64_t i = rlo; i < rhi; ++i) bs[nb++] = r[i].val;           /* r with r.a = a */
        nb = sort_unique(bs, nb);
        for (uint64_t i = 0; i < nb; ++i) {                                   /* s with s.b in B(a) */
            uint64_t lo = lower_key(s, 0, ns, bs[i]), hi = upper_key(s, lo, ns, bs[i]);
            if (!reserve_u32(&cs, &ccap, nc + (hi - lo))) { status = ORC_NOMEM; goto done; }
            for (uint64_t j = lo; j < hi; ++j) cs[nc++] = s[j].val;
        }
        nc = sort_unique(cs, nc);
        for (uint64_t i = 0; i < nc; ++i) {                                   /* t with t.c in C(a) */
            uint64_t lo = lower_key(t, 0, nt, cs[i]), hi = upper_key(t, lo, nt, cs[i]);
            if (!reserve_u32(&ds, &dcap, nd + (hi - lo))) { status = ORC_NOMEM; goto done; }
            for (uint64_t j = lo; j < hi; ++j) ds[nd++] = t[j].val;
        }
        nd = sort_unique(ds, nd);
        uint32_t* sk = sketch + 16 * q;
        for (int j = 0; j < 16; ++j) sk[j] = 0;
        for (uint64_t i = 0; i < nd; ++i) fm_add(sk, ds[i], seed);
        exact[q] = nd;
        est[q] = fm_estimate(sk);
    }
done:
    free(r); free(s); free(t); free(bs); free(cs); free(ds);
    return status;
}

/* The sketch and estimate of an explicit set of values (for the pins). */
int orc_fm_sketch(const uint32_t* vals, uint64_t n, uint32_t seed, uint32_t* sketch, double* est) {
    for (int j = 0; j < 16; ++j) sketch[j] = 0;
    for (uint64_t i = 0; i < n; ++i) fm_add(sketch, vals[i], seed);
    *est = fm_estimate(sketch);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Linear join with its result written out: the materialised form of the    */
/* join of Sec. 4 (Sec. 6's experiments aggregate it instead).  The result   */
/* is the sequence of tuples (a, b, c, d) of R |x| S |x| T in nested-loop    */
/* order: r in R's order; for each r, the s with s.b = r.b in S's order; for */
/* each s, the t with t.c = s.c in T's order.  Bags: every combination of    */
/* matching tuples is one element, duplicates included.                      */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t key; uint32_t pad; uint64_t idx; } kidx_t;

static int cmp_kidx(const void* x, const void* y) {
    const kidx_t* p = (const kidx_t*)x;
    const kidx_t* q = (const kidx_t*)y;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;
    return 0;
}

/* indices of a relation ordered by (key column kcol, position): the tuples */
/* with one key keep the relation's own order                               */
static kidx_t* key_order(const uint32_t* c0, const uint32_t* c1, int64_t stride, uint64_t n, int kcol) {
    kidx_t* p = (kidx_t*)malloc((n ? n : 1) * sizeof(kidx_t));
    if (!p) return NULL;
    for (uint64_t i = 0; i < n; ++i) {
        p[i].key = kcol == 0 ? c0[i * stride] : c1[i * stride];
        p[i].pad = 0;
        p[i].idx = i;
    }
    qsort(p, n, sizeof(kidx_t), cmp_kidx);
    return p;
}

/* [lo, hi) of the entries of p[0, n) with key k */
static void key_range(const kidx_t* p, uint64_t n, uint32_t k, uint64_t* lo, uint64_t* hi) {
    uint64_t a = 0, b = n;
    while (a < b) { uint64_t m = a + (b - a) / 2; if (p[m].key < k) a = m + 1; else b = m; }
    *lo = a;
    b = n;
    while (a < b) { uint64_t m = a + (b - a) / 2; if (p[m].key <= k) a = m + 1; else b = m; }
    *hi = a;
}

/* Elements [lo, lo + cap) of the sequence (those that exist) go to         */
/* out[4 * (pos - lo) ...] as (a, b, c, d); its length goes to *total.        */
int orc_linear3_materialize(const uint32_t* r0, const uint32_t* r1, int64_t rstride, uint64_t nr,
                            const uint32_t* s0, const uint32_t* s1, int64_t sstride, uint64_t ns,
                            const uint32_t* t0, const uint32_t* t1, int64_t tstride, uint64_t nt,
                            uint64_t lo, uint64_t cap, uint32_t* out, uint64_t* total) {
    kidx_t* S = key_order(s0, s1, sstride, ns, 0);   /* S by b */
    kidx_t* T = key_order(t0, t1, tstride, nt, 0);   /* T by c */
    if (!S || !T) { free(S); free(T); return ORC_NOMEM; }
    u128 pos = 0;
    for (uint64_t i = 0; i < nr; ++i) {                                  /* r in R's order */
        const uint32_t a = r0[i * rstride], b = r1[i * rstride];
        uint64_t slo, shi;
        key_range(S, ns, b, &slo, &shi);
        for (uint64_t j = slo; j < shi; ++j) {                           /* s with s.b = b */
            const uint32_t c = s1[S[j].idx * sstride];
            uint64_t tlo, thi;
            key_range(T, nt, c, &tlo, &thi);
            for (uint64_t k = tlo; k < thi; ++k, ++pos) {                /* t with t.c = c */
                if (pos < lo || pos - lo >= cap) continue;
                uint32_t* o = out + 4 * (uint64_t)(pos - lo);
                o[0] = a; o[1] = b; o[2] = c; o[3] = t1[T[k].idx * tstride];
            }
        }
    }
    free(S); free(T);
    if (pos >> 64) return ORC_OVERFLOW;
    *total = (uint64_t)pos;
    return ORC_OK;
}

/* The elements at the positions pos[0, npos) of the same sequence, each     */
/* found from the length of every r's block (the sum over its s of the       */
/* number of t); a position past the end gives (0xFFFFFFFF x 4).  The        */
/* sequence's length goes to *total.                                         */
int orc_linear3_materialize_at(const uint32_t* r0, const uint32_t* r1, int64_t rstride, uint64_t nr,
                               const uint32_t* s0, const uint32_t* s1, int64_t sstride, uint64_t ns,
                               const uint32_t* t0, const uint32_t* t1, int64_t tstride, uint64_t nt,
                               const uint64_t* pos, uint64_t npos, uint32_t* out, uint64_t* total) {
    kidx_t* S = key_order(s0, s1, sstride, ns, 0);
    kidx_t* T = key_order(t0, t1, tstride, nt, 0);
    uint64_t* tdeg = (uint64_t*)malloc((ns ? ns : 1) * sizeof(uint64_t));   /* #t for S[j] */
    uint64_t* start = (uint64_t*)malloc((nr + 1) * sizeof(uint64_t));       /* r's first position */
    int status = ORC_OK;
    if (!S || !T || !tdeg || !start) { status = ORC_NOMEM; goto done; }
    for (uint64_t j = 0; j < ns; ++j) {
        uint64_t tlo, thi;
        key_range(T, nt, s1[S[j].idx * sstride], &tlo, &thi);
        tdeg[j] = thi - tlo;
    }
    u128 acc = 0;
    for (uint64_t i = 0; i < nr; ++i) {
        start[i] = (uint64_t)acc;
        uint64_t slo, shi;
        key_range(S, ns, r1[i * rstride], &slo, &shi);
        for (uint64_t j = slo; j < shi; ++j) acc += tdeg[j];
        if (acc >> 64) { status = ORC_OVERFLOW; goto done; }
    }
    start[nr] = (uint64_t)acc;
    *total = (uint64_t)acc;
    for (uint64_t q = 0; q < npos; ++q) {
        uint32_t* o = out + 4 * q;
        const uint64_t p = pos[q];
        if (p >= start[nr]) { o[0] = o[1] = o[2] = o[3] = 0xFFFFFFFFu; continue; }
        uint64_t a = 0, b = nr;                       /* last r with start[r] <= p */
        while (b - a > 1) { uint64_t m = a + (b - a) / 2; if (start[m] <= p) a = m; else b = m; }
        uint64_t k = p - start[a];
        const uint32_t rb = r1[a * rstride];
        uint64_t slo, shi;
        key_range(S, ns, rb, &slo, &shi);
        for (uint64_t j = slo; j < shi; ++j) {
            if (k >= tdeg[j]) { k -= tdeg[j]; continue; }
            const uint32_t c = s1[S[j].idx * sstride];
            uint64_t tlo, thi;
            key_range(T, nt, c, &tlo, &thi);
            o[0] = r0[a * rstride]; o[1] = rb; o[2] = c; o[3] = t1[T[tlo + k].idx * tstride];
            break;
        }
    }
done:
    free(S); free(T); free(tdeg); free(start);
    return status;
}
