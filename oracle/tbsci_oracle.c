/*
 * tbsci_oracle.c -- plain FP64 CPU reference for the TPB sigma build.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper: Sec. II.A, Eq. TPB_Det and the index map
 * K = (w-1) l_beta + u; Sec. II.C, the Slater-Condon nonzero rule and the six
 * [a,b] categories; Algorithm 1 defines which elements enter sigma):
 *
 *     sigma_K = sum_{L in D_TPB} <D_K|H|D_L> C_L ,   K, L in D_TPB,
 *
 * where D_TPB is every product of a selected alpha string with a selected
 * beta string, C is row-major [l_alpha][l_beta] (beta fastest), and H is the
 * non-relativistic electronic Hamiltonian in a real orthonormal basis,
 *
 *     H = sum_{pq,s} h_pq a+_{ps} a_{qs}
 *       + 1/2 sum_{pqrs,st} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}.
 *
 * The computation is determinant-driven and works in spin orbitals, not in
 * alpha/beta strings: a determinant is one 2M-spin-orbital occupation
 * (alpha orbital p -> spin orbital p, beta orbital p -> spin orbital M+p),
 * ordered as the product of creators in ascending spin-orbital order acting
 * on the vacuum.  For every output determinant the code enumerates every
 * spin-orbital single and double excitation, applies the operators one by
 * one to get the phase, looks the result up in hash tables of the selected
 * strings (excitations leaving the selection are dropped: sigma = P H P C),
 * and evaluates the textbook spin-orbital Slater-Condon element with
 * antisymmetrised integrals <XY||ZW> = <XY|ZW> - <XY|WZ>,
 * <XY|ZW> = (x z|y w) delta(s_X,s_Z) delta(s_Y,s_W).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t cap;      /* power of two */
    uint64_t *key;
    int32_t *val;     /* -1 = empty */
} omap;

static uint64_t mix64(uint64_t x) {
    x ^= x >> 30; x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27; x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

static int omap_init(omap *m, const uint64_t *keys, int64_t n) {
    int64_t cap = 16;
    while (cap < 2 * n + 2) cap <<= 1;
    m->cap = cap;
    m->key = (uint64_t *)malloc(sizeof(uint64_t) * cap);
    m->val = (int32_t *)malloc(sizeof(int32_t) * cap);
    if (!m->key || !m->val) return -1;
    for (int64_t i = 0; i < cap; ++i) m->val[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = (int64_t)(mix64(keys[i]) & (uint64_t)(cap - 1));
        while (m->val[s] >= 0) {
            if (m->key[s] == keys[i]) return -2; /* duplicate */
            s = (s + 1) & (cap - 1);
        }
        m->key[s] = keys[i];
        m->val[s] = (int32_t)i;
    }
    return 0;
}

static int32_t omap_get(const omap *m, uint64_t k) {
    int64_t s = (int64_t)(mix64(k) & (uint64_t)(m->cap - 1));
    while (m->val[s] >= 0) {
        if (m->key[s] == k) return m->val[s];
        s = (s + 1) & (m->cap - 1);
    }
    return -1;
}

static void omap_free(omap *m) { free(m->key); free(m->val); }

typedef struct {
    int M, na, nb;
    int64_t la, lb;
    const double *h, *eri;
    omap amap, bmap;
    /* determinant-level pruning (NULL: every product of a selected alpha and
     * a selected beta string): dmap maps the key ia * lb + ib of each kept
     * determinant to its position in the compact, segment-ordered vector */
    omap *dmap;
} ospace;

/* A determinant in spin orbitals: w[0] = alpha bits, w[1] = beta bits. */
typedef struct { uint64_t w[2]; } det_t;

static int so_occ(const det_t *d, int M, int X) {
    return X < M ? (int)((d->w[0] >> X) & 1u) : (int)((d->w[1] >> (X - M)) & 1u);
}

/* number of occupied spin orbitals with index < X */
static int so_below(const det_t *d, int M, int X) {
    if (X < M) return __builtin_popcountll(d->w[0] & ((X ? (~0ULL >> (64 - X)) : 0ULL)));
    int Y = X - M;
    return __builtin_popcountll(d->w[0]) +
           __builtin_popcountll(d->w[1] & ((Y ? (~0ULL >> (64 - Y)) : 0ULL)));
}

static void so_flip(det_t *d, int M, int X) {
    if (X < M) d->w[0] ^= (1ULL << X); else d->w[1] ^= (1ULL << (X - M));
}

/* apply a_X (create=0) or a+_X (create=1); returns 0 if the result vanishes */
static int so_apply(det_t *d, int M, int X, int create, int *sign) {
    int occ = so_occ(d, M, X);
    if (create == occ) return 0;
    if (so_below(d, M, X) & 1) *sign = -*sign;
    so_flip(d, M, X);
    return 1;
}

/* spin-orbital one-electron integral */
static double h_so(const ospace *s, int X, int Y) {
    int M = s->M;
    if ((X < M) != (Y < M)) return 0.0;
    return s->h[(X % M) * M + (Y % M)];
}

/* physicist <XY|ZW> = (x z | y w) delta(sX,sZ) delta(sY,sW) */
static double g_so(const ospace *s, int X, int Y, int Z, int W) {
    int M = s->M;
    if ((X < M) != (Z < M) || (Y < M) != (W < M)) return 0.0;
    int x = X % M, y = Y % M, z = Z % M, w = W % M;
    return s->eri[(((size_t)x * M + z) * M + y) * M + w];
}

static double g_anti(const ospace *s, int X, int Y, int Z, int W) {
    return g_so(s, X, Y, Z, W) - g_so(s, X, Y, W, Z);
}

static int occ_list(const det_t *d, int M, int *occ) {
    int n = 0;
    for (int X = 0; X < 2 * M; ++X) if (so_occ(d, M, X)) occ[n++] = X;
    return n;
}

static double diag_element(const ospace *s, const det_t *d) {
    int occ[128];
    int n = occ_list(d, s->M, occ);
    double e = 0.0;
    for (int a = 0; a < n; ++a) e += h_so(s, occ[a], occ[a]);
    double g = 0.0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) g += g_anti(s, occ[a], occ[b], occ[a], occ[b]);
    return e + 0.5 * g;
}

/* <a+_A a_X D | H | D> / sign, with D occupied list occ[0..n) */
static double single_element(const ospace *s, const int *occ, int n, int X, int A) {
    double v = h_so(s, A, X);
    for (int k = 0; k < n; ++k) v += g_anti(s, A, occ[k], X, occ[k]);
    return v;
}

static int64_t lookup_det(const ospace *s, const det_t *d, int64_t *col) {
    int32_t ia = omap_get(&s->amap, d->w[0]);
    if (ia < 0) return -1;
    int32_t ib = omap_get(&s->bmap, d->w[1]);
    if (ib < 0) return -1;
    *col = ib;
    return ia;
}

/* C rows supplied through a map: row_slot[ia] = row of Csub holding C[ia, :],
 * or -1 if that row was not supplied (then *missing is set).  With dmap, C
 * is a compact vector over the kept determinants and a determinant that is
 * not kept contributes nothing. */
typedef struct {
    const double *C;
    const int64_t *row_slot; /* NULL: C is the full matrix */
    int *missing;
    const omap *dmap;        /* non-NULL: compact C over the kept determinants */
} cview;

static double cget(const cview *v, int64_t ja, int64_t jb, int64_t lb) {
    if (v->dmap) {
        int32_t k = omap_get(v->dmap, (uint64_t)(ja * lb + jb));
        return k < 0 ? 0.0 : v->C[k];
    }
    if (!v->row_slot) return v->C[ja * lb + jb];
    int64_t r = v->row_slot[ja];
    if (r < 0) {
        *v->missing = 1;
        return 0.0;
    }
    return v->C[r * lb + jb];
}

/* sigma for one output determinant (row ia, column ib) */
static double sigma_one(const ospace *s, const cview *C, int64_t ia, int64_t ib,
                        const uint64_t *alpha, const uint64_t *beta) {
    int M = s->M;
    det_t D; D.w[0] = alpha[ia]; D.w[1] = beta[ib];
    int occ[128], vir[128];
    int n = occ_list(&D, M, occ);
    int nv = 0;
    for (int X = 0; X < 2 * M; ++X) if (!so_occ(&D, M, X)) vir[nv++] = X;
    const int64_t lb = s->lb;
    double acc = diag_element(s, &D) * cget(C, ia, ib, lb);
    /* singles X -> A (same spin only; other spins give zero elements) */
    for (int x = 0; x < n; ++x) {
        for (int a = 0; a < nv; ++a) {
            int X = occ[x], A = vir[a];
            if ((X < M) != (A < M)) continue;
            det_t E = D; int sg = 1;
            so_apply(&E, M, X, 0, &sg);
            so_apply(&E, M, A, 1, &sg);
            int64_t jb, ja = lookup_det(s, &E, &jb);
            if (ja < 0) continue;
            acc += sg * single_element(s, occ, n, X, A) * cget(C, ja, jb, lb);
        }
    }
    /* doubles X<Y -> A<B */
    for (int x = 0; x < n; ++x)
        for (int y = x + 1; y < n; ++y)
            for (int a = 0; a < nv; ++a)
                for (int b = a + 1; b < nv; ++b) {
                    int X = occ[x], Y = occ[y], A = vir[a], B = vir[b];
                    int nxa = (X < M) + (Y < M), naa = (A < M) + (B < M);
                    if (nxa != naa) continue; /* spin changing: zero */
                    double v = g_anti(s, A, B, X, Y);
                    if (v == 0.0) continue;
                    det_t E = D; int sg = 1;
                    so_apply(&E, M, X, 0, &sg);
                    so_apply(&E, M, Y, 0, &sg);
                    so_apply(&E, M, B, 1, &sg);
                    so_apply(&E, M, A, 1, &sg);
                    int64_t jb, ja = lookup_det(s, &E, &jb);
                    if (ja < 0) continue;
                    acc += sg * v * cget(C, ja, jb, lb);
                }
    return acc;
}

/* ---------------------------------------------------------------- API */

void *orc_space_new(int M, int na, int nb, const double *h, const double *eri,
                    const uint64_t *alpha, int64_t la, const uint64_t *beta, int64_t lb,
                    int *status) {
    ospace *s = (ospace *)calloc(1, sizeof(ospace));
    s->M = M; s->na = na; s->nb = nb; s->la = la; s->lb = lb; s->h = h; s->eri = eri;
    *status = 0;
    if (omap_init(&s->amap, alpha, la) || omap_init(&s->bmap, beta, lb)) *status = -1;
    return s;
}

void orc_space_free(void *p) {
    ospace *s = (ospace *)p;
    if (!s) return;
    omap_free(&s->amap); omap_free(&s->bmap);
    if (s->dmap) { omap_free(s->dmap); free(s->dmap); }
    free(s);
}

/*
 * Determinant-level pruning (Sec. II.A, the TBSCI space): row w keeps the
 * beta strings beta_idx[row_off[w] .. row_off[w+1]), and the compact CI
 * vector lists the kept determinants row by row in that order.  Returns 0,
 * or -1 on a malformed layout (offsets not nondecreasing from 0, an index
 * outside [0, l_beta), a repeated index within a row).
 */
int orc_set_dets(void *p, const int64_t *row_off, const int32_t *beta_idx) {
    ospace *s = (ospace *)p;
    if (row_off[0] != 0) return -1;
    int64_t n = row_off[s->la];
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t w = 0; w < s->la; ++w) {
        if (row_off[w + 1] < row_off[w]) { free(keys); return -1; }
        for (int64_t k = row_off[w]; k < row_off[w + 1]; ++k) {
            if (beta_idx[k] < 0 || beta_idx[k] >= s->lb) { free(keys); return -1; }
            keys[k] = (uint64_t)(w * s->lb + beta_idx[k]);
        }
    }
    omap *m = (omap *)calloc(1, sizeof(omap));
    int rc = omap_init(m, keys, n);
    free(keys);
    if (rc) { omap_free(m); free(m); return -1; }
    if (s->dmap) { omap_free(s->dmap); free(s->dmap); }
    s->dmap = m;
    return 0;
}

/*
 * sigma over the kept determinants (Algorithm 1 with both membership
 * tests: an output determinant (w, u) is kept, and so is every connected
 * (x, v) that contributes).  C and out are compact vectors of
 * row_off[l_alpha] entries; (ia, ib) of entry t come from the row layout.
 */
void orc_sigma_dets(void *p, const uint64_t *alpha, const uint64_t *beta, const int64_t *row_off,
                    const int32_t *beta_idx, const double *C, double *out, const int64_t *rows,
                    int64_t nrows, int nthreads) {
    /* rows == NULL: every kept determinant, out in compact order; else only
     * the segments of the listed alpha rows, concatenated in list order */
    ospace *s = (ospace *)p;
    int missing = 0;
    cview v = {C, NULL, &missing, s->dmap};
    int64_t nr = rows ? nrows : s->la;
    int64_t *dst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr + 1));
    dst[0] = 0;
    for (int64_t r = 0; r < nr; ++r) {
        int64_t w = rows ? rows[r] : r;
        dst[r + 1] = dst[r] + row_off[w + 1] - row_off[w];
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t r = 0; r < nr; ++r) {
        int64_t w = rows ? rows[r] : r;
        for (int64_t k = row_off[w]; k < row_off[w + 1]; ++k)
            out[dst[r] + k - row_off[w]] = sigma_one(s, &v, w, beta_idx[k], alpha, beta);
    }
    free(dst);
}

/* sigma rows: rows == NULL -> all alpha rows; out is [nrows][lb] */
static void sigma_rows(ospace *s, const uint64_t *alpha, const uint64_t *beta, const cview *v,
                       double *out, const int64_t *rows, int64_t nrows, int nthreads) {
    int64_t nr = rows ? nrows : s->la;
    int64_t total = nr * s->lb;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t t = 0; t < total; ++t) {
        int64_t r = t / s->lb, ib = t % s->lb;
        int64_t ia = rows ? rows[r] : r;
        out[t] = sigma_one(s, v, ia, ib, alpha, beta);
    }
}

void orc_sigma(void *p, const uint64_t *alpha, const uint64_t *beta, const double *C,
               double *out, const int64_t *rows, int64_t nrows, int nthreads) {
    int missing = 0;
    cview v = {C, NULL, &missing, NULL};
    sigma_rows((ospace *)p, alpha, beta, &v, out, rows, nrows, nthreads);
}

/* As orc_sigma, with C given only for some rows: Csub[row_slot[ia]][:] = C[ia][:].
 * Returns 0, or -1 if an output row needed a C row that was not supplied. */
int orc_sigma_rowmap(void *p, const uint64_t *alpha, const uint64_t *beta, const double *Csub,
                     const int64_t *row_slot, double *out, const int64_t *rows, int64_t nrows,
                     int nthreads) {
    int missing = 0;
    cview v = {Csub, row_slot, &missing, NULL};
    sigma_rows((ospace *)p, alpha, beta, &v, out, rows, nrows, nthreads);
    return missing ? -1 : 0;
}

/* <D_I|H|D_J> for arbitrary determinants (generic Slater-Condon). */
double orc_element(void *p, uint64_t ia_str, uint64_t ib_str, uint64_t ja_str, uint64_t jb_str) {
    ospace *s = (ospace *)p;
    int M = s->M;
    det_t I = {{ia_str, ib_str}}, J = {{ja_str, jb_str}};
    int da = __builtin_popcountll(ia_str ^ ja_str), db = __builtin_popcountll(ib_str ^ jb_str);
    int deg = (da + db) / 2;
    if (deg == 0) return diag_element(s, &I);
    if (deg > 2) return 0.0;
    /* orbitals in J not in I (annihilated from J), in I not in J (created) */
    int ann[4], cre[4], na = 0, nc = 0;
    for (int X = 0; X < 2 * M; ++X) {
        int oi = so_occ(&I, M, X), oj = so_occ(&J, M, X);
        if (oj && !oi) ann[na++] = X;
        if (oi && !oj) cre[nc++] = X;
    }
    if (na != nc) return 0.0;
    if (deg == 1) {
        det_t E = J; int sg = 1;
        so_apply(&E, M, ann[0], 0, &sg);
        so_apply(&E, M, cre[0], 1, &sg);
        int occ[128]; int n = occ_list(&J, M, occ);
        return sg * single_element(s, occ, n, ann[0], cre[0]);
    }
    det_t E = J; int sg = 1;
    so_apply(&E, M, ann[0], 0, &sg);
    so_apply(&E, M, ann[1], 0, &sg);
    so_apply(&E, M, cre[1], 1, &sg);
    so_apply(&E, M, cre[0], 1, &sg);
    return sg * g_anti(s, cre[0], cre[1], ann[0], ann[1]);
}

/* Dense P H P over the whole TPB space, [la*lb][la*lb] row-major. */
void orc_dense(void *p, const uint64_t *alpha, const uint64_t *beta, double *H, int nthreads) {
    ospace *s = (ospace *)p;
    int64_t n = s->la * s->lb;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t K = 0; K < n; ++K) {
        int64_t ia = K / s->lb, ib = K % s->lb;
        for (int64_t L = 0; L < n; ++L) {
            int64_t ja = L / s->lb, jb = L % s->lb;
            H[K * n + L] = orc_element(p, alpha[ia], beta[ib], alpha[ja], beta[jb]);
        }
    }
}

/* Dense P H P over the kept determinants of a TBSCI layout, [n][n]. */
void orc_dense_dets(void *p, const uint64_t *alpha, const uint64_t *beta, const int64_t *row_off,
                    const int32_t *beta_idx, double *H, int nthreads) {
    ospace *s = (ospace *)p;
    int64_t n = row_off[s->la];
    int64_t *wa = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t w = 0; w < s->la; ++w)
        for (int64_t k = row_off[w]; k < row_off[w + 1]; ++k) wa[k] = w;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t K = 0; K < n; ++K)
        for (int64_t L = 0; L < n; ++L)
            H[K * n + L] = orc_element(p, alpha[wa[K]], beta[beta_idx[K]], alpha[wa[L]],
                                       beta[beta_idx[L]]);
    free(wa);
}

/* Diagonal H_KK for selected rows (rows NULL -> all), [nrows][lb]. */
void orc_diag(void *p, const uint64_t *alpha, const uint64_t *beta, double *out,
              const int64_t *rows, int64_t nrows, int nthreads) {
    ospace *s = (ospace *)p;
    int64_t nr = rows ? nrows : s->la;
    int64_t total = nr * s->lb;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t t = 0; t < total; ++t) {
        int64_t r = t / s->lb, ib = t % s->lb;
        int64_t ia = rows ? rows[r] : r;
        det_t D = {{alpha[ia], beta[ib]}};
        out[t] = diag_element(s, &D);
    }
}

/*
 * Excitation lists of one spin by pair scan (independent of any
 * candidate-enumeration scheme): for every selected string I and every
 * selected string J, the excitation degree is popcount(I^J)/2.  Degree 1 and
 * degree 2 pairs are kept; orbitals and phase come from applying, to J, the
 * operator that turns it into I, one creator/annihilator at a time.
 *   kind 1: singles, entry (j, p, q, sign) with I = a+_p a_q J, p in I, q in J
 *           (diag entries p = q are NOT produced here);
 *   kind 2: doubles, entry (j, i, jj, a, b, sign) with i<jj removed from I and
 *           a<b added to I, sign = <I| a+_i a+_jj a_b a_a |J>.
 * Output per row is in the canonical order: singles by (p, q), doubles by
 * (i, jj, a, b).  count_only != 0 just counts entries.
 * Rows are given by row indices (rows NULL -> all).  Returns total entries;
 * row_ptr has nrows+1 entries; ent is int32 [total][6] (j, o0, o1, o2, o3, sign).
 */
static int apply_str(uint64_t *s, int X, int create, int *sign) {
    int occ = (int)((*s >> X) & 1u);
    if (create == occ) return 0;
    if (__builtin_popcountll(*s & (X ? (~0ULL >> (64 - X)) : 0ULL)) & 1) *sign = -*sign;
    *s ^= (1ULL << X);
    return 1;
}

int64_t orc_lists(const uint64_t *str, int64_t l, int M, int kind, const int64_t *rows,
                  int64_t nrows, int64_t *row_ptr, int32_t *ent, int count_only) {
    int64_t nr = rows ? nrows : l;
    int64_t tot = 0;
    for (int64_t r = 0; r < nr; ++r) {
        int64_t ii = rows ? rows[r] : r;
        uint64_t I = str[ii];
        row_ptr[r] = tot;
        int64_t start = tot;
        for (int64_t jj = 0; jj < l; ++jj) {
            uint64_t J = str[jj];
            int d = __builtin_popcountll(I ^ J) / 2;
            if (d != kind) continue;
            uint64_t rem = I & ~J, add = J & ~I; /* rem: in I only; add: in J only */
            int o[4]; int sg = 1; uint64_t s = J;
            if (kind == 1) {
                int p = __builtin_ctzll(rem), q = __builtin_ctzll(add);
                apply_str(&s, q, 0, &sg);
                apply_str(&s, p, 1, &sg);
                o[0] = p; o[1] = q; o[2] = o[3] = 0;
            } else {
                int i = __builtin_ctzll(rem), j2 = 63 - __builtin_clzll(rem);
                int a = __builtin_ctzll(add), b = 63 - __builtin_clzll(add);
                /* I = a+_i a+_j2 a_b a_a J : apply right to left */
                apply_str(&s, a, 0, &sg);
                apply_str(&s, b, 0, &sg);
                apply_str(&s, j2, 1, &sg);
                apply_str(&s, i, 1, &sg);
                o[0] = i; o[1] = j2; o[2] = a; o[3] = b;
            }
            if (!count_only) {
                int32_t *e = ent + 6 * tot;
                e[0] = (int32_t)jj; e[1] = o[0]; e[2] = o[1]; e[3] = o[2]; e[4] = o[3]; e[5] = sg;
            }
            ++tot;
        }
        if (!count_only) {
            /* insertion sort of the row by its orbital key */
            int64_t n = tot - start;
            int32_t *base = ent + 6 * start;
            for (int64_t x = 1; x < n; ++x) {
                int32_t t[6]; memcpy(t, base + 6 * x, sizeof t);
                int64_t kt = ((int64_t)t[1] << 24) | ((int64_t)t[2] << 16) | (t[3] << 8) | t[4];
                int64_t y = x - 1;
                while (y >= 0) {
                    int32_t *u = base + 6 * y;
                    int64_t ku = ((int64_t)u[1] << 24) | ((int64_t)u[2] << 16) | (u[3] << 8) | u[4];
                    if (ku <= kt) break;
                    memcpy(base + 6 * (y + 1), u, sizeof t);
                    --y;
                }
                memcpy(base + 6 * (y + 1), t, sizeof t);
            }
        }
    }
    row_ptr[nr] = tot;
    return tot;
}

/*
 * Single-excitation entry count of a complete or selected list by candidate
 * enumeration with hash membership (used to reproduce the link-table sizes
 * of the paper's memory-footprint table without storing the table).
 */
int64_t orc_count_singles(const uint64_t *str, int64_t l, int M, int nthreads) {
    omap m;
    if (omap_init(&m, str, l)) return -1;
    int64_t tot = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for reduction(+ : tot) schedule(static)
#endif
    for (int64_t i = 0; i < l; ++i) {
        uint64_t I = str[i];
        for (int q = 0; q < M; ++q) {
            if (!((I >> q) & 1u)) continue;
            for (int p = 0; p < M; ++p) {
                if ((I >> p) & 1u) continue;
                if (omap_get(&m, (I ^ (1ULL << q)) | (1ULL << p)) >= 0) ++tot;
            }
        }
    }
    omap_free(&m);
    return tot;
}
