/*
 * Fast CPU oracle: the thesis's own CPU method for the symmetrized H.v.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: nothing in the product library
 * links, loads or calls this file, and it shares no code with the HIP
 * library.  It exists so that the oracle can run whole matrix-vector
 * products and Lanczos runs at sizes where the brute-force orbits of
 * oracle.c take hours (36 sites), with its own independent code.
 *
 * Method (thesis, section "Sublattice Coding techniques"):
 *   - the sites split into n_sub sublattices of b = n / n_sub consecutive
 *     sites, sublattice 0 on the most significant bits; every group element
 *     maps each sublattice onto a sublattice (sublattice stability, checked
 *     here);
 *   - lookup tables, algorithm "Preparation of lookup tables for sublattice
 *     coding": for every sublattice X and substate s,
 *       SymmetryAction_X(g, s) = g|s>_X as a full 64-bit configuration (spin
 *         flip included: the bits of the image sublattice are reversed),
 *       G_X = { g : g maps sublattice X onto sublattice 0 },
 *       Rep_X(s) = min over g in G_X of int(g|s>_X),
 *       Sym_X(s) = { g in G_X : g|s>_X = Rep_X(s) };
 *   - algorithm "Sublattice coding algorithm for finding the
 *     representative": MinRep = min_X Rep_X(sigma_X); every g in Sym_Y of a
 *     sublattice Y attaining MinRep is applied by OR-ing its
 *     SymmetryAction_X over all X, and the smallest image is the
 *     representative.  Every minimizing g is among these candidates and each
 *     g is a candidate once (it maps exactly one sublattice onto sublattice
 *     0), so the number of minimizers is |Stab|, and chi is trivial on the
 *     stabilizer iff every minimizer has the same character;
 *   - basis: the sector's configurations in ascending order, kept iff their
 *     own representative with chi trivial on the stabilizer; configurations
 *     are visited substate by substate, and a prefix is dropped as soon as
 *     one of its sublattices X has Rep_X below the leading substate (some g
 *     then maps the configuration below itself);
 *   - H.v in the pull form of oracle.c (orc_rows), with the pieces of
 *     orc_apply_terms (those with equal targets merged), the index found by
 *     binary search inside the range that a table of limits on the leading
 *     bits gives; OpenMP over rows.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef struct {
    int n, n_sub, b, G;
    uint64_t S;            /* 2^b substates per sublattice */
    uint64_t *act;         /* [n_sub][G][S]: SymmetryAction_X(g, s) */
    uint64_t *rep;         /* [n_sub][S]: Rep_X(s), as a full configuration (sublattice 0's bits) */
    int64_t *sym_off;      /* [n_sub * S + 1] */
    int32_t *sym;          /* Sym_X(s) lists: group elements */
    const double *chi_re, *chi_im;
} orf_tables;

static inline uint64_t bit_of_site(int n, int site) { return (uint64_t)1 << (n - 1 - site); }

/* substate s of sublattice X placed into a configuration (bit k of s is
 * site X*b + b-1-k) */
static inline uint64_t place(const orf_tables *t, int X, uint64_t s) { return s << (t->n - (X + 1) * t->b); }
static inline uint64_t substate(const orf_tables *t, uint64_t c, int X)
{
    return (c >> (t->n - (X + 1) * t->b)) & (t->S - 1);
}

void orf_free(orf_tables *t)
{
    if (!t) return;
    free(t->act);
    free(t->rep);
    free(t->sym_off);
    free(t->sym);
    free(t);
}

/* Tables for n_sub sublattices; NULL if a group element splits a sublattice
 * or the tables would be too large. */
orf_tables *orf_build(const orc_problem *p, int n_sub)
{
    const int n = p->n, G = p->n_elem;
    if (n_sub < 1 || n % n_sub) return NULL;
    const int b = n / n_sub;
    if (b > 20) return NULL;
    const uint64_t S = (uint64_t)1 << b;
    if ((double)n_sub * G * (double)S * 8.0 > 4.0e9) return NULL;
    /* image sublattice of every (g, X); -1: not stable */
    int *img = malloc(sizeof(int) * (size_t)G * n_sub);
    if (!img) return NULL;
    for (int g = 0; g < G; ++g)
        for (int X = 0; X < n_sub; ++X) {
            const int32_t *pm = p->perm + (size_t)g * n;
            const int Y = pm[X * b] / b;
            for (int i = X * b; i < (X + 1) * b; ++i)
                if (pm[i] / b != Y) { free(img); return NULL; }
            img[g * n_sub + X] = Y;
        }
    orf_tables *t = calloc(1, sizeof(orf_tables));
    if (!t) { free(img); return NULL; }
    t->n = n; t->n_sub = n_sub; t->b = b; t->G = G; t->S = S; t->chi_re = p->chi_re; t->chi_im = p->chi_im;
    t->act = malloc(sizeof(uint64_t) * (size_t)n_sub * G * S);
    t->rep = malloc(sizeof(uint64_t) * (size_t)n_sub * S);
    t->sym_off = malloc(sizeof(int64_t) * ((size_t)n_sub * S + 1));
    int64_t *cnt = calloc((size_t)n_sub * S + 1, sizeof(int64_t));
    if (!t->act || !t->rep || !t->sym_off || !cnt) { free(cnt); free(img); orf_free(t); return NULL; }
    /* SymmetryAction: the spin of site i goes to site perm[i], reversed when g flips */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int X = 0; X < n_sub; ++X)
        for (int g = 0; g < G; ++g) {
            const int32_t *pm = p->perm + (size_t)g * n;
            uint64_t *out = t->act + ((size_t)X * G + g) * S;
            for (uint64_t s = 0; s < S; ++s) {
                const uint64_t c = place(t, X, s);
                uint64_t v = 0;
                for (int i = X * b; i < (X + 1) * b; ++i) {
                    const int up = (c & bit_of_site(n, i)) != 0;
                    if (up != (p->flip[g] != 0)) v |= bit_of_site(n, pm[i]);
                }
                out[s] = v;
            }
        }
    /* Rep and the sizes of the Sym lists */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int X = 0; X < n_sub; ++X)
        for (uint64_t s = 0; s < S; ++s) {
            uint64_t best = ~(uint64_t)0;
            int64_t k = 0;
            for (int g = 0; g < G; ++g) {
                if (img[g * n_sub + X] != 0) continue;
                const uint64_t v = t->act[((size_t)X * G + g) * S + s];
                if (v < best) { best = v; k = 1; } else if (v == best) ++k;
            }
            t->rep[(size_t)X * S + s] = best;
            cnt[(size_t)X * S + s + 1] = k;
        }
    for (uint64_t q = 0; q < (uint64_t)n_sub * S; ++q) cnt[q + 1] += cnt[q];
    memcpy(t->sym_off, cnt, sizeof(int64_t) * ((size_t)n_sub * S + 1));
    t->sym = malloc(sizeof(int32_t) * (size_t)(cnt[(size_t)n_sub * S] + 1));
    if (!t->sym) { free(cnt); free(img); orf_free(t); return NULL; }
    #pragma omp parallel for collapse(2) schedule(static)
    for (int X = 0; X < n_sub; ++X)
        for (uint64_t s = 0; s < S; ++s) {
            int64_t k = t->sym_off[(size_t)X * S + s];
            for (int g = 0; g < G; ++g)
                if (img[g * n_sub + X] == 0 && t->act[((size_t)X * G + g) * S + s] == t->rep[(size_t)X * S + s])
                    t->sym[k++] = g;
        }
    free(cnt);
    free(img);
    return t;
}

/* Rep_X(s) as a b-bit substate, and the Sym_X(s) list (up to cap entries;
 * returns its length) */
uint64_t orf_rep_of(const orf_tables *t, int X, uint64_t s)
{
    return t->rep[(size_t)X * t->S + s] >> (t->n - t->b);
}

int orf_sym_of(const orf_tables *t, int X, uint64_t s, int32_t *out, int cap)
{
    const int64_t a = t->sym_off[(size_t)X * t->S + s], e = t->sym_off[(size_t)X * t->S + s + 1];
    for (int64_t q = a; q < e && q - a < cap; ++q) out[q - a] = t->sym[q];
    return (int)(e - a);
}

/* representative of c, the first minimizing element g0, |Stab| and whether
 * chi is trivial on the stabilizer of c.  The minimizers are g0 Stab(c), so
 * chi is trivial on Stab(c) iff every minimizer has the character of g0
 * (compared to 1e-6: distinct roots of unity of order <= |G| lie much
 * further apart). */
void orf_find_rep(const orf_tables *t, uint64_t c, uint64_t *rep, int32_t *g_min, int32_t *stab, int32_t *triv)
{
    uint64_t minrep = ~(uint64_t)0;
    for (int X = 0; X < t->n_sub; ++X) {
        const uint64_t r = t->rep[(size_t)X * t->S + substate(t, c, X)];
        if (r < minrep) minrep = r;
    }
    uint64_t best = ~(uint64_t)0;
    int32_t bg = -1, k = 0, tv = 1;
    for (int Y = 0; Y < t->n_sub; ++Y) {
        const uint64_t sy = substate(t, c, Y);
        if (t->rep[(size_t)Y * t->S + sy] != minrep) continue;
        for (int64_t q = t->sym_off[(size_t)Y * t->S + sy]; q < t->sym_off[(size_t)Y * t->S + sy + 1]; ++q) {
            const int g = t->sym[q];
            uint64_t v = 0;
            for (int X = 0; X < t->n_sub; ++X) v |= t->act[((size_t)X * t->G + g) * t->S + substate(t, c, X)];
            if (v < best) {
                best = v; bg = g; k = 1; tv = 1;
            } else if (v == best) {
                ++k;
                if (fabs(t->chi_re[g] - t->chi_re[bg]) + fabs(t->chi_im[g] - t->chi_im[bg]) > 1e-6) tv = 0;
            }
        }
    }
    *rep = best; *g_min = bg; *stab = k; *triv = tv;
}

void orf_find_rep_many(const orf_tables *t, const uint64_t *c, int64_t m, uint64_t *rep, int32_t *g_min,
                       int32_t *stab, int8_t *triv)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        int32_t g, st, tv;
        orf_find_rep(t, c[i], &rep[i], &g, &st, &tv);
        if (g_min) g_min[i] = g;
        if (stab) stab[i] = st;
        if (triv) triv[i] = (int8_t)tv;
    }
}

/*
 * Sector basis with n_up up spins, ascending.  The configurations are
 * visited sublattice by sublattice (substates ascending, so configurations
 * ascending), with the leading substate s0 fixed per task:
 *   - Rep_0(s0) must be s0 itself (the identity is in G_0);
 *   - a later sublattice X with Rep_X(s_X) below s0's image drops the
 *     prefix: some g in G_X maps the configuration below itself.
 * A configuration that survives is checked by orf_find_rep.  Pass 1 counts
 * per leading substate, pass 2 writes (when reps is not NULL and the
 * dimension fits cap).  Returns the dimension, or -1 without memory for the
 * counts.
 */
typedef struct {
    const orf_tables *t;
    int n_up;
    uint64_t lead;         /* s0 placed at sublattice 0 */
    uint64_t *reps;        /* NULL: count only */
    int32_t *stabs;
    int64_t k;
} orf_walk;

static int popc(uint64_t v) { return __builtin_popcountll(v); }

static void walk(orf_walk *w, int X, uint64_t prefix, int left)
{
    const orf_tables *t = w->t;
    if (X == t->n_sub) {
        if (left) return;
        uint64_t r; int32_t g, st, tv;
        orf_find_rep(t, prefix, &r, &g, &st, &tv);
        if (r == prefix && tv) {
            if (w->reps) { w->reps[w->k] = prefix; if (w->stabs) w->stabs[w->k] = st; }
            ++w->k;
        }
        return;
    }
    const int rest = (t->n_sub - 1 - X) * t->b;   /* bits after sublattice X */
    for (uint64_t s = 0; s < t->S; ++s) {
        const int pc = popc(s);
        if (pc > left || left - pc > rest) continue;
        if (t->rep[(size_t)X * t->S + s] < w->lead) continue;
        walk(w, X + 1, prefix | place(t, X, s), left - pc);
    }
}

int64_t orf_enumerate(const orf_tables *t, int n_up, uint64_t *reps, int32_t *stabs, int64_t cap)
{
    const uint64_t S = t->S;
    int64_t *cnt = calloc(S + 1, sizeof(int64_t));
    if (!cnt) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (uint64_t s0 = 0; s0 < S; ++s0) {
        const int pc = popc(s0);
        if (pc > n_up || n_up - pc > t->n - t->b) continue;
        if (t->rep[s0] != place(t, 0, s0)) continue;
        orf_walk w = {t, n_up, place(t, 0, s0), NULL, NULL, 0};
        walk(&w, 1, place(t, 0, s0), n_up - pc);
        cnt[s0 + 1] = w.k;
    }
    for (uint64_t q = 0; q < S; ++q) cnt[q + 1] += cnt[q];
    const int64_t dim = cnt[S];
    if (reps && dim <= cap) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (uint64_t s0 = 0; s0 < S; ++s0) {
            if (cnt[s0 + 1] == cnt[s0]) continue;
            orf_walk w = {t, n_up, place(t, 0, s0), reps + cnt[s0], stabs ? stabs + cnt[s0] : NULL, 0};
            walk(&w, 1, place(t, 0, s0), n_up - popc(s0));
        }
    }
    free(cnt);
    return dim;
}

/*
 * Index of a representative through a table of limits on its leading bits
 * (the thesis's "Limits" lookup of its distributed-memory section): the
 * representatives with leading P bits equal to q occupy positions
 * [lim[q], lim[q + 1]) of the ascending basis, and a binary search runs
 * inside that range only.  -1 if absent.
 */
typedef struct {
    int shift;             /* n - P */
    int64_t *lim;          /* [2^P + 1] */
} orf_limits;

static orf_limits limits_build(const uint64_t *reps, int64_t dim, int n)
{
    orf_limits L;
    const int P = n < 22 ? n : 22;
    const uint64_t Q = (uint64_t)1 << P;
    L.shift = n - P;
    L.lim = malloc(sizeof(int64_t) * (Q + 1));
    if (!L.lim) return L;
    int64_t i = 0;
    for (uint64_t q = 0; q <= Q; ++q) {
        while (i < dim && (reps[i] >> L.shift) < q) ++i;
        L.lim[q] = i;
    }
    return L;
}

static int64_t limits_find(const orf_limits *L, const uint64_t *reps, uint64_t s)
{
    const uint64_t q = s >> L->shift;
    const int64_t j = orc_find(reps + L->lim[q], L->lim[q + 1] - L->lim[q], s);
    return j < 0 ? -1 : L->lim[q] + j;
}

/*
 * Pieces of one row with equal targets, their amplitudes summed (the
 * non-branching terms that flip the same pair of spins, e.g. an exchange and
 * the chirality terms on that bond, act as one term with the summed
 * amplitude): a small open-addressing table keyed by the target, emptied per
 * row by a generation count.
 */
typedef struct {
    int mask;
    uint64_t *key;
    int32_t *slot;         /* position in the merged list */
    uint32_t *gen;
    uint32_t cur;
} orf_merge;

static int merge_init(orf_merge *M, int mt)
{
    int size = 16;
    while (size < 2 * mt) size <<= 1;
    M->mask = size - 1;
    M->key = malloc(sizeof(uint64_t) * size);
    M->slot = malloc(sizeof(int32_t) * size);
    M->gen = calloc(size, sizeof(uint32_t));
    M->cur = 0;
    return M->key && M->slot && M->gen;
}

static void merge_free(orf_merge *M)
{
    free(M->key);
    free(M->slot);
    free(M->gen);
}

/* merges the m pieces (tau, h) in place; returns the number of distinct targets */
static int merge_pieces(orf_merge *M, uint64_t *tau, double complex *h, int m)
{
    if (++M->cur == 0) {                 /* generation wrapped: clear */
        memset(M->gen, 0, sizeof(uint32_t) * (size_t)(M->mask + 1));
        M->cur = 1;
    }
    int u = 0;
    for (int q = 0; q < m; ++q) {
        uint64_t k = tau[q] * 0x9E3779B97F4A7C15ull;
        int e = (int)(k >> 40) & M->mask;
        while (M->gen[e] == M->cur && M->key[e] != tau[q]) e = (e + 1) & M->mask;
        if (M->gen[e] == M->cur) {
            h[M->slot[e]] += h[q];
        } else {
            M->gen[e] = M->cur;
            M->key[e] = tau[q];
            M->slot[e] = u;
            tau[u] = tau[q];
            h[u] = h[q];
            ++u;
        }
    }
    return u;
}

/*
 * y = H x over the whole basis, pull form (as orc_rows):
 *   y_i = sum_k chi(g) sqrt(|Stab tau~| / |Stab sigma_i|) conj(h_k) x(tau~_k)
 * over the pieces of orc_apply_terms whose target lies in the basis, pieces
 * with equal targets merged first.  x, y: interleaved complex (re, im) when
 * cplx, else real.  Returns 0, or -1 when the table of limits or a merge
 * table cannot be allocated (y untouched).
 */
int orf_apply(const orc_problem *p, const orf_tables *t, const uint64_t *reps, const int32_t *stabs, int64_t dim,
               const double *x, double *y, int cplx)
{
    const int mt = orc_max_terms(p);
    orf_limits lim = limits_build(reps, dim, t->n);
    if (!lim.lim) return -1;
    int failed = 0;
    #pragma omp parallel
    {
        uint64_t *tau = malloc(sizeof(uint64_t) * mt);
        double complex *h = malloc(sizeof(double complex) * mt);
        orf_merge M;
        const int ok = merge_init(&M, mt) && tau && h;
        #pragma omp atomic
        failed += !ok;
        #pragma omp barrier
        if (!failed) {
            #pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < dim; ++i) {
                const int m = merge_pieces(&M, tau, h, orc_apply_terms(p, reps[i], tau, h));
                double complex acc = 0;
                for (int q = 0; q < m; ++q) {
                    if (h[q] == 0) continue;
                    uint64_t r; int32_t g, st, tv;
                    orf_find_rep(t, tau[q], &r, &g, &st, &tv);
                    if (!tv) continue;
                    const int64_t j = limits_find(&lim, reps, r);
                    if (j < 0) continue;
                    const double complex chi = p->chi_re[g] + I * p->chi_im[g];
                    const double complex c = chi * sqrt((double)st / (double)stabs[i]) * conj(h[q]);
                    const double complex xj = cplx ? x[2 * j] + I * x[2 * j + 1] : x[j];
                    acc += c * xj;
                }
                if (cplx) { y[2 * i] = creal(acc); y[2 * i + 1] = cimag(acc); }
                else y[i] = creal(acc);
            }
        }
        free(tau);
        free(h);
        merge_free(&M);
    }
    free(lim.lim);
    return failed ? -1 : 0;
}
