/*
 * symed — matrix-free Hamiltonian application in a symmetry-adapted basis
 * for spin-1/2 lattice models, on one AMD Instinct MI355X (gfx950).
 *
 * Plain C ABI: host/device pointers and sizes only.  Streams are HIP streams
 * (hipStream_t) passed as `void*`; NULL means the default stream.  Every
 * call returns an ed_status; no C++ exception crosses this boundary.  On
 * error the outputs are left untouched and ed_last_error() returns a
 * thread-local message describing the failure.
 *
 * Conventions (thesis chapter on large-scale exact diagonalization):
 *  - A configuration of N <= 63 spins is an N-bit integer: site 0 is the
 *    most significant bit, spin up = 1 (eq. defining int(sigma) in
 *    "Representing Hilbert spaces and operators").
 *  - A group element g moves the spin at site i to site perm[g*N + i]; if
 *    flip[g] != 0 every spin is reversed afterwards.  The group must be
 *    closed under composition and chi a one-dimensional character of it
 *    (1-D irreps only, section "Computations in the symmetrized basis").
 *  - Basis states are orbit representatives: the smallest integer in the
 *    orbit ("representative condition").  A representative belongs to the
 *    sector iff chi is trivial on its stabilizer.  Basis order = ascending
 *    integer value.
 *  - Sites are labelled so that each sublattice is a contiguous block of
 *    N/N_sub labels, sublattice 0 on the most significant bits (section
 *    "Generic sublattice coding algorithm": site numbering); every group
 *    element must map each block onto one block (sublattice stability).
 *  - Vectors are contiguous float64 arrays of length dim, or interleaved
 *    complex128 (re, im) when the sector is complex (complex characters or
 *    chirality terms).  Vectors are caller-owned device memory.
 */
#ifndef SYMED_H
#define SYMED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ED_OK = 0,
    ED_EINVAL = 1,        /* bad argument, inconsistent model/group, H not invariant */
    ED_ENOTSTABLE = 2,    /* sublattice decomposition not stable under the group */
    ED_ECHAR = 3,         /* characters not a 1-D representation (|chi|!=1 or not multiplicative) */
    ED_ENOMEM = 4,        /* device or host allocation failed, or memory cap exceeded */
    ED_EDEVICE = 5,       /* HIP runtime error */
    ED_EBREAKDOWN = 6     /* Lanczos breakdown: beta vanished before n_iter steps */
} ed_status;

/* Thread-local description of the last failure (never NULL). */
const char *ed_last_error(void);

/* Library version string. */
const char *ed_version(void);

/*
 * Hamiltonian H = sum_b J_b S_i.S_j + sum_t Jchi_t S_i.(S_j x S_k)
 * (Heisenberg bonds as in the thesis's model chapters; scalar chirality on
 * oriented triangles, as in the J1-J2-Jchi triangular model).  Every term is
 * decomposed into non-branching pieces (section "Computations in the
 * symmetrized basis"); pieces flipping the same pair of sites are merged.
 *   bond_sites: int32[n_bonds][2], bond_J: f64[n_bonds]
 *   tri_sites:  int32[n_tri][3] (i,j,k), tri_Jchi: f64[n_tri]
 * Host pointers, read during ed_basis_build only.
 */
typedef struct {
    int32_t n_sites;
    int32_t n_bonds;
    const int32_t *bond_sites;
    const double *bond_J;
    int32_t n_tri;
    const int32_t *tri_sites;
    const double *tri_Jchi;
} ed_model;

/*
 * Symmetry group and 1-D irrep: perm int32[n_elem][n_sites], flip
 * uint8[n_elem], chi_re/chi_im f64[n_elem] (chi_im may be NULL for real
 * characters).  Host pointers, read during ed_basis_build only.
 * n_elem <= 65535.  Spin-flip elements require n_up == n_sites/2.
 */
typedef struct {
    int32_t n_elem;
    const int32_t *perm;
    const uint8_t *flip;
    const double *chi_re;
    const double *chi_im;
} ed_group;

/*
 * Build options.  Zero means "choose automatically".
 *  n_sub_rep:   sublattices of the Rep/Sym lookup tables (sublattice coding).
 *  n_sub_act:   sublattices of the SymmetryAction tables; a multiple of
 *               n_sub_rep (a refinement in the same contiguous labelling).
 *  prefix_bits: bits of the Limits prefix table of the plain index lookup.
 *  mem_limit_bytes: cap on the device memory owned by the basis together
 *               with the temporaries of the calls working on it while they
 *               are held (0 = none); exceeding it fails with ED_ENOMEM.
 */
typedef struct {
    int32_t n_sub_rep;
    int32_t n_sub_act;
    int32_t prefix_bits;
    int32_t reserved;
    int64_t mem_limit_bytes;
} ed_options;

typedef struct ed_basis ed_basis;

typedef struct {
    int64_t dim;               /* sector dimension */
    int32_t is_complex;        /* vectors are complex128 */
    int32_t n_sites;
    int32_t n_elem;
    int32_t n_sub_rep, n_sub_act, prefix_bits;
    int64_t n_elements;        /* matrix entries evaluated per H.v: the diagonal of
                                  every row plus every (row, flipped pair) with
                                  non-zero amplitude, in sector or not */
    int64_t n_offdiag;         /* n_elements - dim */
    int64_t bytes_device;      /* device memory owned by the basis */
    int64_t table_bytes;       /* sublattice-coding tables (resident in LDS) */
    int64_t limits_bytes;      /* plain lookup prefix table */
    int64_t index_bytes;       /* learned index: network, segment and cell tables (0 if not trained) */
    int32_t index_max_err;     /* learned index: largest search window (-1 if not trained) */
    int32_t lds_resident;      /* tables staged in LDS by the kernels */
    double build_seconds;      /* wall time of ed_basis_build */
    double limits_mean_window; /* plain lookup: mean Limits bucket over all keys */
    int64_t limits_max_window; /* plain lookup: largest Limits bucket */
    int32_t apply_blocks;      /* persistent grid of the H.v kernel */
    int32_t apply_threads;     /* its block size */
    int32_t n_colors;          /* SU(d) bases: d; spin-1/2 bases: 0 */
    int32_t reserved;
} ed_basis_info_t;

/*
 * Build the sector basis on the device: validate model, group, characters
 * and sublattice stability; build the sublattice-coding tables (Rep, Sym,
 * SymmetryAction; algorithm "Preparation of lookup tables"); enumerate the
 * Sz sector and keep representatives whose stabilizer carries a trivial
 * character (algorithm "Preparation of the distributed and symmetrized
 * Hilbert space", on one device); build the Limits prefix table.
 *   n_up: number of up spins (Sz sector).
 *   stream: hipStream_t or NULL.  Blocks until the basis is complete.
 *   out: receives a library-owned handle; free with ed_basis_free.
 * Errors: ED_EINVAL, ED_ENOTSTABLE, ED_ECHAR, ED_ENOMEM, ED_EDEVICE.
 */
ed_status ed_basis_build(const ed_model *model, const ed_group *group, int32_t n_up,
                         const ed_options *opts, void *stream, ed_basis **out);

/*
 * SU(d) permutation model in a color-count sector (thesis, chapter on SU(N)
 * chiral spin liquids, the SU(N) Heisenberg model with imaginary ring
 * exchange on elementary triangles):
 *     H = sum_b J_b P_ij + sum_t K_t i (P_ijk - P_ijk^-1),
 * P_ij exchanging the colors of sites i and j, P_ijk moving the color of i to
 * j, of j to k and of k to i.  The model struct is read with that meaning:
 * bond_J are the exchange couplings J_b, tri_Jchi the ring couplings K_t of the
 * oriented triangles tri_sites.  For d = 2, P_ij = 2 S_i.S_j + 1/2 and
 * i (P_ijk - P_ijk^-1) = 4 S_i.(S_j x S_k).
 *   n_colors: d in [2, 4]; counts: int32[n_colors] (host), the number of
 *   sites of each color, adding up to n_sites <= 31.
 * A site holds its color in two bits: a configuration is the integer
 * sum_i color_i 4^(n_sites-1-i) (site 0 most significant).  The group (no
 * spin-flip elements) acts on sites; representatives, stabilizers, norms,
 * basis order, sublattice stability and vectors follow the spin-1/2
 * conventions above, read on these integers.  ed_options counts sublattices
 * as for spin-1/2 bases (a sublattice of m sites is a 2m-bit substate);
 * prefix_bits counts bits of the 2 n_sites-bit keys.
 * The returned basis works with ed_apply_H, ed_lookup, ed_hash_build,
 * ed_lanczos_*, ed_basis_info/export/device_reps (lookup modes 0 and 2);
 * ed_index_train, the spin-1/2 observables (ed_apply_op*, ed_expectation)
 * and batches reject it with ED_EINVAL.
 * Errors: as ed_basis_build; ED_EINVAL also for counts that do not add up to
 * n_sites, flip elements, or more than 2^58 configurations in the sector.
 */
ed_status ed_basis_build_colors(const ed_model *model, const ed_group *group, int32_t n_colors, const int32_t *counts,
                                const ed_options *opts, void *stream, ed_basis **out);

/* Release everything the basis owns (tables, representatives, indexes,
 * captured graphs).  NULL is ignored. */
void ed_basis_free(ed_basis *basis);

/* Sizes and statistics of a built basis. */
ed_status ed_basis_info(const ed_basis *basis, ed_basis_info_t *info);

/*
 * Copy the basis to the host: reps uint64[dim] (ascending representatives),
 * stab uint32[dim] (stabilizer sizes; norm N = sqrt(|G| |Stab|)).
 * Either pointer may be NULL.  Synchronous.
 */
ed_status ed_basis_export(const ed_basis *basis, uint64_t *h_reps, uint32_t *h_stab);

/* Device pointer to the ascending representatives (uint64[dim]), owned by
 * the basis and valid until ed_basis_free. */
ed_status ed_basis_device_reps(const ed_basis *basis, const uint64_t **d_reps);

/*
 * y := H x in the symmetry-adapted basis (matrix-free; algorithm "Parallel
 * matrix-vector multiply for a non-branching term", as a gather: each row's
 * owner applies every non-branching piece to its representative, finds the
 * target's representative by sublattice coding (algorithm "Sublattice coding
 * algorithm for finding the representative"), looks up its index, and
 * accumulates character x norm ratio x amplitude x x_j; no atomics).
 *   d_x, d_y: device vectors of length dim (f64 or interleaved c128); must
 *   not alias.  lookup_mode: 0 = plain (Limits + binary search), 1 = learned
 *   index (requires ed_index_train; in real sectors x is first copied into
 *   the index's {representative, x} records), 2 = hashed staging table
 *   (requires ed_hash_build; x is first copied into the table).  The basis
 *   owns those records, so calls with mode 1 or 2 on one basis must not
 *   overlap in time.  The result is the same in every mode, bit for bit.
 *   Asynchronous on `stream`.
 */
ed_status ed_apply_H(const ed_basis *basis, const void *d_x, void *d_y, int32_t lookup_mode, void *stream);

/*
 * Index lookup of n representatives: d_idx[k] = position of d_keys[k] in the
 * basis, or -1 if absent.  mode 0 = plain (Limits + binary search), 1 =
 * learned index + bounded search, 2 = membership from the hashed table
 * (positions then from the plain lookup).  d_keys uint64[n], d_idx int64[n] device
 * memory.  Asynchronous on `stream`.
 */
ed_status ed_lookup(const ed_basis *basis, const uint64_t *d_keys, int64_t n, int64_t *d_idx,
                    int32_t mode, void *stream);

/*
 * Lanczos iteration without reorthogonalization (algorithms "Real-symmetric
 * Lanczos step" and "Complex-Hermitian Lanczos step"), n_iter steps from the
 * start vector d_v0 (device, length dim; normalized internally, not
 * modified).  Each step is one replay of a captured HIP graph (H.v with the
 * fused w <- Hv - beta w epilogue, reductions, axpy, scale) with alpha and
 * beta kept on the device.  Results: h_alpha f64[n_iter], h_beta f64[n_iter]
 * (beta[k] is the norm produced by step k; the T-matrix off-diagonal is
 * beta[0..n-2]); *n_done = steps completed.  Returns ED_EBREAKDOWN (with
 * outputs valid for n_done steps) if beta < 1e-14 max|alpha|.
 * lookup_mode as in ed_apply_H.  Blocks until done.
 */
ed_status ed_lanczos_run(const ed_basis *basis, const void *d_v0, int32_t n_iter, int32_t lookup_mode,
                         double *h_alpha, double *h_beta, int32_t *n_done, void *stream);

/*
 * Ground-state vectors and expectation values (thesis, "The Lanczos
 * algorithm": the eigenvectors of T give the Ritz vectors, and a second
 * Lanczos run from the same start vector rebuilds them from the Lanczos
 * vectors without storing those).
 *
 * ed_ritz_vector: k-th lowest eigenvalue (*lambda, may be NULL) and the
 *   normalized eigenvector coef[n] of T (diagonal alpha[n], off-diagonal
 *   beta[n-1]); Sturm bisection, then inverse iteration.  Host only.
 * ed_lanczos_vector: repeats n_iter steps from d_v0 (as ed_lanczos_run,
 *   same lookup_mode) and writes d_psi = sum_k coef[k] v_k, normalized
 *   (device vector like d_v0, must not alias it).  Blocks until done.
 * ed_expectation: <psi|O|psi> for an operator O of the same form as H
 *   (bonds J S_i.S_j and chirality triangles), which must be invariant
 *   under the basis's group (checked; ED_EINVAL otherwise).  O's pair table
 *   replaces H's in the H.v kernel; the result's real part goes to *re and
 *   the imaginary part (0 up to rounding for Hermitian O; complex sectors
 *   only) to *im (may be NULL).  Allocates a vector of dim entries
 *   temporarily.  Blocks until done.
 * ed_apply_op: d_y := O d_x for such an operator (same checks) and, when
 *   d_z is not NULL, <z, y> = sum_i conj(z_i) y_i to *re and *im (im: complex
 *   sectors; may be NULL).  Two calls give <psi|A B|psi> = <A psi, B psi>
 *   for Hermitian invariant A and B: the four-spin bond-bond and six-spin
 *   chirality-chirality correlations of the thesis's order parameters
 *   (chapter on the triangular J1-J2-Jchi model, nematic and chirality
 *   order parameters).  Vectors as in ed_apply_H (caller-owned, dim
 *   entries, y must not alias x; z may be x, y or another vector);
 *   lookup_mode 1 and 2 stage x into the basis's records, so calls on one
 *   basis must not overlap.  Allocates O's tables temporarily.  Blocks
 *   until done.
 * On an empty sector (dim 0) ed_expectation and ed_apply_op return ED_OK at
 *   once with *re = *im = 0, before the operator is checked.
 */
ed_status ed_ritz_vector(const double *alpha, const double *beta, int32_t n, int32_t k, double *lambda,
                         double *coef);
ed_status ed_lanczos_vector(const ed_basis *basis, const void *d_v0, int32_t n_iter, int32_t lookup_mode,
                            const double *h_coef, void *d_psi, void *stream);
ed_status ed_expectation(const ed_basis *basis, const ed_model *op, const void *d_psi, int32_t lookup_mode,
                         double *re, double *im, void *stream);
ed_status ed_apply_op(const ed_basis *basis, const ed_model *op, const void *d_x, void *d_y, const void *d_z,
                      int32_t lookup_mode, double *re, double *im, void *stream);

/*
 * ed_apply_op without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same y := O x and <z, y> as
 * ed_apply_op, with the same arguments, checks and results, but the
 * operator's tables (at most 224 KiB) and the dot partials (at most 32 KiB)
 * live in a static 256 KiB device array of the library instead of
 * temporaries.  Each device the library runs on holds its own copy of that
 * array until the process ends; its address is looked up at the first call
 * on a device.  The basis must live on the current device.  All calls on one
 * device share the array and leave their contents in it: calls of this
 * entry point that overlap in time on one device race (as do mode 1 and 2
 * calls on one basis, see ed_apply_H).  Tables larger than the array fail
 * with ED_EINVAL before anything runs.  Blocks until done.
 */
ed_status ed_apply_op_noalloc(const ed_basis *basis, const ed_model *op, const void *d_x, void *d_y,
                              const void *d_z, int32_t lookup_mode, double *re, double *im, void *stream);

/*
 * Hashed staging table (not in the thesis).  The gather needs, for every
 * target, only x at the target's position.  This table holds records
 * {representative, x} (real) or {representative, Re x, Im x, unused}
 * (complex) in `slots` = dim / load slots, placed by linear probing from a
 * hash of the representative (MurmurHash3's 64-bit finalizer, reduced by a
 * multiply-high).  Before each H.v in lookup_mode 2 the input vector is
 * copied into the records; a lookup then probes from the home slot, and the
 * line that confirms the key also holds x_j.  Memory: slots x 16 (real) or
 * 32 (complex) bytes plus 4 bytes per state.  load: fraction of occupied
 * slots, in [0.05, 0.95]; 0 = default: 0.15 (real sectors) or 0.25
 * (complex sectors), or the smallest load in hundredths that keeps the slot
 * count below 4e9.  Needs n_sites < 64.  A second
 * call with the same load returns the stats; another load is refused.
 * Blocks until built.
 */
typedef struct {
    double load;
    int32_t reserved[2];
} ed_hash_cfg;

typedef struct {
    int64_t slots;
    int64_t bytes;             /* table + position-to-slot map */
    double load;               /* dim / slots */
    double mean_probes;        /* slots visited to find a representative, mean over the basis */
    int64_t max_probes;
    double build_seconds;
} ed_hash_stats;

ed_status ed_hash_build(ed_basis *basis, const ed_hash_cfg *cfg, ed_hash_stats *stats, void *stream);

/*
 * n_more further steps of the last ed_lanczos_run on this basis (any
 * available lookup_mode: the steps are the same bit for bit), from the
 * device state it left; h_alpha, h_beta: f64[n_more] for the new steps only;
 * *n_done = new steps completed.  A run and its resumptions give exactly the
 * coefficients of one run of the total length, so convergence can be
 * checked between chunks.  ED_EINVAL if there is no run to resume (none
 * yet, or ed_lanczos_vector ran since); ED_EBREAKDOWN if the run broke
 * down.  Blocks until done.
 */
ed_status ed_lanczos_resume(const ed_basis *basis, int32_t n_more, int32_t lookup_mode, double *h_alpha,
                            double *h_beta, int32_t *n_done, void *stream);

/*
 * Lowest k eigenvalues of the symmetric tridiagonal T-matrix with diagonal
 * alpha[n] and off-diagonal beta[n-1] (Sturm-sequence bisection), ascending.
 * Host only.
 */
ed_status ed_eigenvalues(const double *alpha, const double *beta, int32_t n, int32_t k, double *evals);

/*
 * Learned index over the ascending representative list (not in the thesis;
 * measured against its "Limits" prefix map, section on distributed-memory
 * parallelization, which stays the plain lookup and the reference).
 *  - Input: the rank of the key among all N-bit configurations with the
 *    sector's number of up spins, in ascending order (combinatorial number
 *    system), read as a fraction u of the largest rank in the basis.
 *  - Network: 1 -> 32 -> 32 -> 1, float32 weights (half of each hidden layer
 *    relu(z), half min(z,0); weights kept non-negative, so the network is
 *    non-decreasing).  Trained on the device with the library's own forward,
 *    backward and Adam kernels on minibatches of (key, position) pairs, then
 *    expanded exactly into its linear pieces (at most 1090), which lookups
 *    evaluate from LDS.  Its output picks one of 2^log2_segments segments.
 *  - Segment: maps the rank linearly onto its cells; cells are allocated in
 *    proportion to the keys routed to the segment (about keys_per_cell each).
 *  - Cell: the position range [first, first + n) of its keys, a prediction
 *    by linear interpolation inside the cell, and its recorded largest
 *    errors below and above the prediction.  Segments whose cells need a
 *    wider window than max_window get four times the cells, a few rounds at
 *    most.
 *  - Lookup: rank -> network -> segment -> cell -> prediction; the search
 *    starts at the predicted position and stays inside the recorded window,
 *    so every representative is found and every other key reported absent:
 *    the lookups agree exactly with the plain Limits + binary search.
 * routing selects what picks the segment: 0 = the trained network, 1 = the
 * network at its initial weights (no training step), 2 = no network (the
 * segment is the feature u itself); the tables below are built the same way,
 * so the three can be compared.  Zero fields mean defaults (n_features = 1
 * and hidden = 32, the only values accepted; steps = 3000, batch = 8192, lr =
 * 1e-2 with cosine decay; log2_segments ~ log2(dim / 2048) within [4, 22];
 * keys_per_cell = 64; max_window = 16).
 */
typedef struct {
    int32_t n_features;
    int32_t hidden;
    int32_t steps;
    int32_t batch;
    float lr;
    uint32_t seed;
    int32_t log2_segments;
    int32_t keys_per_cell;
    int32_t max_window;
    int32_t routing;
} ed_index_cfg;

typedef struct {
    int32_t max_err;           /* largest search window of a representative (keys) */
    int32_t n_segments;
    float final_loss;          /* last minibatch mean squared error (normalized positions) */
    float mlp_max_err;         /* max |network estimate * dim - position| over all keys */
    int64_t mlp_bytes;         /* network weights (float32) */
    int64_t table_bytes;       /* segment and cell tables */
    double train_seconds;      /* training + table build wall time */
    double mean_window;        /* mean search window over all representatives (keys) */
    int32_t n_features;        /* network inputs (1) */
    int32_t n_pieces;          /* linear pieces of the network */
    int64_t used_segments;     /* segments with at least one key */
    float feature_offset;      /* network input x = (u - feature_offset) * feature_scale */
    float feature_scale;
    int64_t n_cells;
    int64_t refined_segments;  /* segments given more cells to meet max_window */
    double mean_abs_err;       /* mean |predicted - true position| */
    double frac_exact;         /* representatives whose prediction is their position */
    double mean_lines;         /* mean 128-byte lines of 16-byte records spanned by the window */
    int64_t lds_bytes;         /* expanded network and rank table (staged in LDS) */
    int32_t routing;
    int32_t reserved;
} ed_index_stats;

/*
 * Train the learned index of a built basis (device kernels; blocks until
 * done) and build its segment and cell tables.  Real sectors also get a
 * record {representative, x} per state in basis order (16 B per state), from
 * which the mode-1 H.v gather reads x_j.  Afterwards lookup_mode / mode 1 is
 * accepted by ed_apply_H, ed_lookup and ed_lanczos_run.  Training again
 * replaces the index.  Temporaries count against the basis's memory cap.
 * Errors: ED_EINVAL, ED_ENOMEM, ED_EDEVICE.
 */
ed_status ed_index_train(ed_basis *basis, const ed_index_cfg *cfg, ed_index_stats *out, void *stream);

/* Statistics of the trained index; h_params (may be NULL) receives the
 * float32 weights W1[32][F], b1[32], W2[32][32], b2[32], W3[32], b3 when
 * cap is large enough.  ED_EINVAL if no index was trained. */
ed_status ed_index_info(const ed_basis *basis, ed_index_stats *out, float *h_params, int64_t cap);

/*
 * Evaluate the trained index network (expanded form) on n keys: d_u[k] =
 * input feature of d_keys[k], d_y[k] = network output (NaN for both when the
 * key is not a configuration of the sector: wrong number of up spins or bits
 * at or above N).  Device pointers (uint64[n], float32[n], float32[n]);
 * asynchronous on `stream`.
 */
ed_status ed_index_predict(const ed_basis *basis, const uint64_t *d_keys, int64_t n, float *d_u, float *d_y,
                           void *stream);

/*
 * Loss and gradient of the index network on an explicit batch, computed by
 * the same forward/backward kernels as training (used to verify them):
 * loss = (1/2n) sum_s (f(X_s) - t_s)^2 (any 1 <= n_features <= 8; no weight
 * projection).  d_params: float32 weights as in
 * ed_index_info; d_X: float32[n][n_features] features; d_t: float32[n];
 * d_grad: float32[#params]; d_loss: float32[1].  All device pointers.
 * Blocks until done.
 */
ed_status ed_mlp_loss_grad(int32_t n_features, const float *d_params, const float *d_X, const float *d_t, int64_t n,
                           float *d_grad, float *d_loss, void *stream);

/*
 * Many sectors in one persistent launch.  A batch references built bases
 * (which must outlive it) and runs H.v, or whole Lanczos steps, for all of
 * them at once: the rows of all sectors are cut into equal tiles, every
 * block of one persistent grid walks the tiles round-robin and stages the
 * tables of a tile's sector into LDS when it changes sector.  One Lanczos
 * step of all sectors is captured once as a HIP graph and replayed.  Real
 * and complex sectors may be mixed; lookup_mode 1 needs a trained learned
 * index in every sector, lookup_mode 2 the hashed staging table in every
 * sector (the input vectors are copied into the tables first, so mode-2
 * calls must not overlap with other calls on those sectors).
 *
 * Launch shape: the tile length and the blocks per compute unit of the
 * persistent grid.  With autotune (the default when tile_rows is 0), the
 * first call in a lookup mode times one batched H.v in that mode for every
 * candidate (tile lengths 2048, 8192 and 32768 rows, with one block per
 * compute unit or as many as fit) and keeps the fastest for that mode.  With
 * cache_path, choices are looked up in that text file first and appended to
 * it after a tuning, keyed by a fingerprint of the batch (device, lookup
 * mode, and every sector's dimension, group order, element count,
 * decompositions and table size): a later batch of the same sectors reuses
 * them without timing.  Each sector's rows are always summed by one lane in
 * term order, so H.v does not depend on the launch shape; the Lanczos
 * reductions are summed per tile, so their rounding does (a cached choice
 * reproduces the tuned run bit for bit).  Concurrent writers of one cache
 * file are not coordinated.
 */
typedef struct ed_batch ed_batch;

typedef struct {
    int32_t tile_rows;          /* fixed tile length (used with autotune = 0) */
    int32_t autotune;
    int32_t blocks_per_cu;      /* fixed blocks per compute unit (0: as many as fit) */
    int32_t reserved;
    const char *cache_path;     /* tuning cache file, or NULL */
} ed_batch_cfg;

typedef struct {
    int32_t n_sectors;
    int32_t tile_rows;          /* tile length in use */
    int64_t n_tiles;
    int64_t total_dim;
    int64_t total_elements;     /* matrix entries evaluated per batched H.v */
    int32_t apply_blocks;       /* persistent grid in use */
    int32_t n_candidates;       /* candidates timed by the last tuning (0: none) */
    int32_t tune_rows[8];
    int32_t tune_blocks[8];     /* blocks per compute unit of each candidate */
    double tune_seconds[8];     /* one batched H.v per candidate */
    int32_t tune_mode;          /* lookup mode of the last choice (-1: none) */
    int32_t cache_hit;          /* the last choice came from the cache file */
    int32_t blocks_per_cu;      /* in use */
    int32_t reserved;
} ed_batch_info_t;

/* Create a batch of n sectors (n <= 256); stream: hipStream_t or NULL.
 * Allocates Lanczos vectors for every sector; blocks until set up. */
ed_status ed_batch_create(ed_basis *const *sectors, int32_t n, const ed_batch_cfg *cfg, void *stream,
                          ed_batch **out);

/* y_s := H_s x_s for every sector s in one launch; d_x, d_y: host arrays of
 * n device vector pointers (layout as ed_apply_H).  Asynchronous on stream. */
ed_status ed_batch_apply(ed_batch *batch, const void *const *d_x, void *const *d_y, int32_t lookup_mode,
                         void *stream);

/* n_iter Lanczos steps of every sector from start vectors d_v0[s]; h_alpha,
 * h_beta: f64[n][n_iter] (sector-major); n_done: int32[n].  Returns
 * ED_EBREAKDOWN if any sector broke down (its n_done < n_iter). */
ed_status ed_batch_lanczos(ed_batch *batch, const void *const *d_v0, int32_t n_iter, int32_t lookup_mode,
                           double *h_alpha, double *h_beta, int32_t *n_done, void *stream);

ed_status ed_batch_info(const ed_batch *batch, ed_batch_info_t *info);

/* Release the batch (not its sectors).  NULL is ignored. */
void ed_batch_free(ed_batch *batch);

/*
 * Decomposition tuner.  The representative does not depend on the
 * sublattice decomposition (any admissible pair gives the same basis), but
 * the cost of the search does.  For every pair (n_sub_rep, n_sub_act) of
 * stable contiguous decompositions with n_sub_rep dividing n_sub_act (at
 * most 16 pairs, finest first), build the sector, prepare lookup_mode
 * (trained index or hashed table with default settings), time one H.v after
 * a warm-up, free it, and return the fastest pair.  Pairs the build refuses
 * (tables too large) are reported with a time of -1.  With cache_path a
 * stored choice (same model, group, characters, Sz sector, lookup mode and
 * device) is returned without timing, and a new choice is appended.
 * Blocks until done; allocates and frees device memory.
 */
typedef struct {
    int32_t n_candidates;
    int32_t cache_hit;
    int32_t sub_rep[16];
    int32_t sub_act[16];
    double seconds[16];
} ed_tune_report;

ed_status ed_tune_decomposition(const ed_model *model, const ed_group *group, int32_t n_up, int32_t lookup_mode,
                                const char *cache_path, void *stream, int32_t *n_sub_rep, int32_t *n_sub_act,
                                ed_tune_report *report);

/*
 * Host-only inspection of the sublattice-coding tables for one
 * decomposition into n_sub contiguous sublattices (no device needed):
 * for sublattice X and substate s (b = N/n_sub bits),
 *   rep_out[X*2^b + s]      = Rep_X(s)
 *   sym_off[X*2^b + s .. +1] = range in sym_out of Sym_X(s) (group indices)
 *   act_out[(g*n_sub + X)*2^b + s] = SymmetryAction_X(g, s) as an N-bit
 *                              configuration (may be NULL)
 * Sizes: rep_out uint32[n_sub*2^b], sym_off uint32[n_sub*2^b + 1],
 * sym_out uint32[sym_cap], act_out uint64[n_elem*n_sub*2^b].
 * *n_sym receives the total length of the Sym lists (sym_out written only
 * if it fits sym_cap).  Validates group and stability as ed_basis_build.
 */
ed_status ed_tables_inspect(const ed_model *model, const ed_group *group, int32_t n_up, int32_t n_sub,
                            uint32_t *rep_out, uint32_t *sym_off, uint32_t *sym_out, int64_t sym_cap,
                            int64_t *n_sym, uint64_t *act_out);

#ifdef __cplusplus
}
#endif

#endif /* SYMED_H */
