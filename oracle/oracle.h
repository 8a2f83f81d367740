/*
 * Shared declarations of the CPU oracle (test infrastructure only; see
 * oracle.c).  The problem description: a spin-1/2 model of bonds and
 * oriented triangles, and a group of site permutations with spin flip and a
 * one-dimensional character.
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <complex.h>
#include <stdint.h>

typedef struct {
    int32_t n;                 /* sites */
    int32_t n_elem;            /* group order */
    const int32_t *perm;       /* [n_elem][n] */
    const uint8_t *flip;       /* [n_elem] */
    const double *chi_re;      /* [n_elem] */
    const double *chi_im;
    const uint8_t *chi_one;    /* [n_elem]: 1 iff chi(g) == 1 */
    int32_t n_bonds;
    const int32_t *bonds;      /* [n_bonds][2] */
    const double *bond_J;
    int32_t n_tri;
    const int32_t *tris;       /* [n_tri][3] */
    const double *tri_J;
} orc_problem;

/* every non-branching piece of H on configuration s: (tau, h) pairs; the
 * Ising part comes last as one diagonal piece (tau = s) */
int orc_apply_terms(const orc_problem *p, uint64_t s, uint64_t *tau, double complex *h);
int orc_max_terms(const orc_problem *p);
/* plain binary search in ascending reps; -1 if absent */
int64_t orc_find(const uint64_t *reps, int64_t dim, uint64_t s);

#endif
