/*
 * CPU oracle for symmetrized exact diagonalization of spin-1/2 models.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP library.
 *
 * Everything here is the plain definition, written for obviousness, not
 * speed:
 *   - a group element acts bit by bit: the spin at site i moves to site
 *     perm[i], then all spins are reversed if flip is set (thesis, section
 *     "Discrete symmetries"; site 0 is the most significant bit, up = 1,
 *     eq. for int(sigma) in "Representing Hilbert spaces and operators");
 *   - the representative of sigma is the smallest integer in its orbit and
 *     g_sigma the (first) group element reaching it (eq. "representative
 *     condition", section "Computations in the symmetrized basis");
 *   - brute force over every group element, no sublattice coding;
 *   - a basis state is kept iff it is its own representative and the
 *     character is trivial on its stabilizer (otherwise the projected state
 *     vanishes), with norm N = sqrt(|G| |Stab|);
 *   - matrix elements follow the symmetrized matrix element
 *     <tau~|H_k|sigma~> = conj(chi(g_tau)) N_tau/N_sigma <tau|H_k|sigma~>;
 *     the conjugate comes from the projector convention
 *     sum_g conj(chi(g)) g|sigma> with the site action above;
 *   - index lookup by plain binary search in the ascending basis.
 *
 * Hamiltonian terms, written as non-branching pieces (section "Computations
 * in the symmetrized basis"):
 *   J S_i.S_j = J S^z_i S^z_j + J/2 (S^+_i S^-_j + S^-_i S^+_j)
 *   Jchi S_i.(S_j x S_k) = (i Jchi / 2) sum_cyc S^z_a (S^+_b S^-_c - S^-_b S^+_c)
 * over the cyclic rotations (a,b,c) of the oriented triangle (i,j,k).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static inline int spin_at(uint64_t s, int n, int site) { return (int)((s >> (n - 1 - site)) & 1u); }
static inline uint64_t site_bit(int n, int site) { return (uint64_t)1 << (n - 1 - site); }

/* g|s>: bit by bit */
uint64_t orc_act(int n, const int32_t *perm, int flip, uint64_t s)
{
    uint64_t out = 0;
    for (int i = 0; i < n; ++i)
        if (spin_at(s, n, i)) out |= site_bit(n, perm[i]);
    if (flip) {
        uint64_t mask = (n == 64) ? ~(uint64_t)0 : (((uint64_t)1 << n) - 1);
        out ^= mask;
    }
    return out;
}

/* representative (minimum over the whole orbit), first minimizing element,
 * stabilizer size, and whether chi is trivial on the stabilizer */
void orc_rep(const orc_problem *p, uint64_t s, uint64_t *rep, int32_t *g_min, int32_t *stab, int32_t *chi_triv)
{
    uint64_t best = ~(uint64_t)0;
    int32_t bg = -1, st = 0, triv = 1;
    for (int g = 0; g < p->n_elem; ++g) {
        uint64_t t = orc_act(p->n, p->perm + (size_t)g * p->n, p->flip[g], s);
        if (t < best) { best = t; bg = g; }
        if (t == s) { ++st; if (!p->chi_one[g]) triv = 0; }
    }
    *rep = best; *g_min = bg; *stab = st; *chi_triv = triv;
}

/* k-th (0-based) n-bit integer with `ones` set bits, in ascending order */
static uint64_t binom_u64(int n, int k)
{
    if (k < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    unsigned __int128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (unsigned)(n - k + i) / (unsigned)i;
    return (uint64_t)r;
}

static uint64_t unrank(int n, int ones, uint64_t r)
{
    uint64_t s = 0;
    for (int pos = n - 1; pos >= 0 && ones > 0; --pos) {
        uint64_t c = binom_u64(pos, ones);   /* integers with bit pos clear */
        if (r >= c) { s |= (uint64_t)1 << pos; r -= c; --ones; }
    }
    return s;
}

static inline uint64_t next_same_popcount(uint64_t v)
{
    uint64_t t = v | (v - 1);
    return (t + 1) | (((~t & -~t) - 1) >> (__builtin_ctzll(v) + 1));
}

/* is s its own representative?  (s <= g s for every g; stops at the first
 * counterexample)  If so, stab and chi-triviality are returned as well. */
static int is_rep(const orc_problem *p, uint64_t s, int32_t *stab, int32_t *triv)
{
    int32_t st = 0, tv = 1;
    for (int g = 0; g < p->n_elem; ++g) {
        uint64_t t = orc_act(p->n, p->perm + (size_t)g * p->n, p->flip[g], s);
        if (t < s) return 0;
        if (t == s) { ++st; if (!p->chi_one[g]) tv = 0; }
    }
    *stab = st; *triv = tv;
    return 1;
}

/*
 * Enumerate the basis of the sector: configurations with n_up up spins in
 * ascending order, kept iff representative and chi trivial on the stabilizer.
 * Work is split into nchunk contiguous rank ranges (threads), then
 * concatenated in order, so the result is ascending.
 * Returns the dimension; writes at most cap entries.
 */
int64_t orc_enumerate(const orc_problem *p, int n_up, uint64_t *reps, int32_t *stabs, int64_t cap)
{
    int n = p->n;
    uint64_t total = binom_u64(n, n_up);
    if (total == 0) return 0;
    int nchunk = 1024;
    if ((uint64_t)nchunk > total) nchunk = (int)total;
    int64_t *cnt = calloc((size_t)nchunk + 1, sizeof(int64_t));
    /* pass 1: count */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nchunk; ++c) {
        uint64_t r0 = (uint64_t)((unsigned __int128)total * (unsigned)c / (unsigned)nchunk);
        uint64_t r1 = (uint64_t)((unsigned __int128)total * (unsigned)(c + 1) / (unsigned)nchunk);
        uint64_t s = unrank(n, n_up, r0);
        int64_t k = 0;
        for (uint64_t r = r0; r < r1; ++r) {
            int32_t st, tv;
            if (is_rep(p, s, &st, &tv) && tv) ++k;
            if (r + 1 < r1) s = next_same_popcount(s);
        }
        cnt[c + 1] = k;
    }
    for (int c = 0; c < nchunk; ++c) cnt[c + 1] += cnt[c];
    int64_t dim = cnt[nchunk];
    if (reps && dim <= cap) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int c = 0; c < nchunk; ++c) {
            uint64_t r0 = (uint64_t)((unsigned __int128)total * (unsigned)c / (unsigned)nchunk);
            uint64_t r1 = (uint64_t)((unsigned __int128)total * (unsigned)(c + 1) / (unsigned)nchunk);
            uint64_t s = unrank(n, n_up, r0);
            int64_t k = cnt[c];
            for (uint64_t r = r0; r < r1; ++r) {
                int32_t st, tv;
                if (is_rep(p, s, &st, &tv) && tv) { reps[k] = s; if (stabs) stabs[k] = st; ++k; }
                if (r + 1 < r1) s = next_same_popcount(s);
            }
        }
    }
    free(cnt);
    return dim;
}

/* plain binary search; -1 if absent */
int64_t orc_find(const uint64_t *reps, int64_t dim, uint64_t s)
{
    int64_t lo = 0, hi = dim - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (reps[mid] == s) return mid;
        if (reps[mid] < s) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* all non-branching pieces H_k acting on s: appends (tau, h) pairs, returns count.
 * The Ising part is returned as a single diagonal piece (tau = s). */
int orc_apply_terms(const orc_problem *p, uint64_t s, uint64_t *tau, double complex *h)
{
    int n = p->n, m = 0;
    double diag = 0.0;
    for (int b = 0; b < p->n_bonds; ++b) {
        int i = p->bonds[2 * b], j = p->bonds[2 * b + 1];
        double J = p->bond_J[b];
        int si = spin_at(s, n, i), sj = spin_at(s, n, j);
        diag += J * (si == sj ? 0.25 : -0.25);
        if (si != sj) {
            tau[m] = s ^ site_bit(n, i) ^ site_bit(n, j);
            h[m] = 0.5 * J;
            ++m;
        }
    }
    for (int t = 0; t < p->n_tri; ++t) {
        const int32_t *v = p->tris + 3 * t;
        double J = p->tri_J[t];
        for (int r = 0; r < 3; ++r) {
            int a = v[r], b = v[(r + 1) % 3], c = v[(r + 2) % 3];
            double sza = spin_at(s, n, a) ? 0.5 : -0.5;
            int sb = spin_at(s, n, b), sc = spin_at(s, n, c);
            if (!sb && sc) {            /* S^+_b S^-_c: b down -> up, c up -> down */
                tau[m] = s ^ site_bit(n, b) ^ site_bit(n, c);
                h[m] = I * 0.5 * J * sza;
                ++m;
            } else if (sb && !sc) {     /* - S^-_b S^+_c */
                tau[m] = s ^ site_bit(n, b) ^ site_bit(n, c);
                h[m] = -I * 0.5 * J * sza;
                ++m;
            }
        }
    }
    tau[m] = s; h[m] = diag; ++m;
    return m;
}

int orc_max_terms(const orc_problem *p) { return p->n_bonds + 3 * p->n_tri + 1; }

/*
 * Push form (the definition): for every column j and every piece H_k,
 * H_k|sigma~_j> = h |tau>,  entry (i = index(tau~), j) +=
 * conj(chi(g_tau)) sqrt(|Stab tau|/|Stab sigma_j|) h.
 * Entries for targets outside the basis are dropped.  COO triplets, not
 * merged.  Returns the number of entries (writes at most cap).
 */
int64_t orc_coo(const orc_problem *p, const uint64_t *reps, const int32_t *stabs, int64_t dim,
                int64_t *ri, int64_t *ci, double *vre, double *vim, int64_t cap)
{
    int mt = orc_max_terms(p);
    int64_t *cnt = calloc((size_t)dim + 1, sizeof(int64_t));
    #pragma omp parallel
    {
        uint64_t *tau = malloc(sizeof(uint64_t) * mt);
        double complex *h = malloc(sizeof(double complex) * mt);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t j = 0; j < dim; ++j) {
            int m = orc_apply_terms(p, reps[j], tau, h);
            int64_t k = 0;
            for (int q = 0; q < m; ++q) {
                if (h[q] == 0) continue;
                uint64_t rt; int32_t g, st, tv;
                orc_rep(p, tau[q], &rt, &g, &st, &tv);
                if (tv && orc_find(reps, dim, rt) >= 0) ++k;
            }
            cnt[j + 1] = k;
        }
        #pragma omp single
        for (int64_t j = 0; j < dim; ++j) cnt[j + 1] += cnt[j];
        #pragma omp for schedule(dynamic, 64)
        for (int64_t j = 0; j < dim; ++j) {
            if (cnt[dim] > cap) continue;
            int m = orc_apply_terms(p, reps[j], tau, h);
            int64_t k = cnt[j];
            for (int q = 0; q < m; ++q) {
                if (h[q] == 0) continue;
                uint64_t rt; int32_t g, st, tv;
                orc_rep(p, tau[q], &rt, &g, &st, &tv);
                if (!tv) continue;
                int64_t i = orc_find(reps, dim, rt);
                if (i < 0) continue;
                double complex chi = p->chi_re[g] + I * p->chi_im[g];
                double complex v = conj(chi) * sqrt((double)st / (double)stabs[j]) * h[q];
                ri[k] = i; ci[k] = j; vre[k] = creal(v); vim[k] = cimag(v);
                ++k;
            }
        }
        free(tau); free(h);
    }
    int64_t total = cnt[dim];
    free(cnt);
    return total;
}

/*
 * Pull form for given rows (gather; uses hermiticity H_ij = conj(H_ji)):
 *   y(sigma~_i) = sum_k chi(g_tau) sqrt(|Stab tau|/|Stab sigma_i|) conj(h_k) x(tau~_k)
 * over pieces whose target tau~ lies in the sector (rep with chi trivial on
 * its stabilizer).  Rows must be sector representatives; row_ok[r] = 0
 * flags one that is not.  Output: per row, entries (tau~, coefficient),
 * CSR-like with row_ptr[n_rows+1]; at most cap entries written.
 * Also returns, per row, the number of "elements": the diagonal plus every
 * distinct flipped configuration with non-zero amplitude (in sector or not).
 */
int64_t orc_rows(const orc_problem *p, const uint64_t *rows, int64_t n_rows, int64_t *row_ptr,
                 uint64_t *tgt, double *cre, double *cim, int64_t cap, int8_t *row_ok, int32_t *n_elements)
{
    int mt = orc_max_terms(p);
    row_ptr[0] = 0;
    int64_t *cnt = calloc((size_t)n_rows + 1, sizeof(int64_t));
    #pragma omp parallel
    {
        uint64_t *tau = malloc(sizeof(uint64_t) * mt);
        double complex *h = malloc(sizeof(double complex) * mt);
        #pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n_rows; ++r) {
            uint64_t s = rows[r];
            uint64_t rs; int32_t gs, sts, tvs;
            orc_rep(p, s, &rs, &gs, &sts, &tvs);
            row_ok[r] = (rs == s && tvs) ? 1 : 0;
            int m = orc_apply_terms(p, s, tau, h);
            int64_t k = 0;
            int ne = 0;
            for (int q = 0; q < m; ++q) {
                /* distinct configurations with non-zero summed amplitude */
                int first = 1;
                for (int q2 = 0; q2 < q; ++q2) if (tau[q2] == tau[q]) { first = 0; break; }
                if (first) {
                    double complex acc = 0;
                    for (int q2 = q; q2 < m; ++q2) if (tau[q2] == tau[q]) acc += h[q2];
                    if (acc != 0 || tau[q] == s) ++ne;
                }
                if (h[q] == 0) continue;
                uint64_t rt; int32_t g, st, tv;
                orc_rep(p, tau[q], &rt, &g, &st, &tv);
                if (tv) ++k;
            }
            cnt[r + 1] = k;
            if (n_elements) n_elements[r] = ne;
        }
        #pragma omp single
        for (int64_t r = 0; r < n_rows; ++r) cnt[r + 1] += cnt[r];
        #pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n_rows; ++r) {
            if (cnt[n_rows] > cap) continue;
            uint64_t s = rows[r];
            uint64_t rs; int32_t gs, sts, tvs;
            orc_rep(p, s, &rs, &gs, &sts, &tvs);
            int m = orc_apply_terms(p, s, tau, h);
            int64_t k = cnt[r];
            for (int q = 0; q < m; ++q) {
                if (h[q] == 0) continue;
                uint64_t rt; int32_t g, st, tv;
                orc_rep(p, tau[q], &rt, &g, &st, &tv);
                if (!tv) continue;
                double complex chi = p->chi_re[g] + I * p->chi_im[g];
                double complex v = chi * sqrt((double)st / (double)sts) * conj(h[q]);
                tgt[k] = rt; cre[k] = creal(v); cim[k] = cimag(v);
                ++k;
            }
        }
        free(tau); free(h);
    }
    for (int64_t r = 0; r <= n_rows; ++r) row_ptr[r] = cnt[r];
    int64_t total = cnt[n_rows];
    free(cnt);
    return total;
}

/* batch representative computation */
void orc_rep_many(const orc_problem *p, const uint64_t *s, int64_t n, uint64_t *rep, int32_t *g_min,
                  int32_t *stab, int8_t *chi_triv)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int32_t g, st, tv;
        orc_rep(p, s[i], &rep[i], &g, &st, &tv);
        if (g_min) g_min[i] = g;
        if (stab) stab[i] = st;
        if (chi_triv) chi_triv[i] = (int8_t)tv;
    }
}
