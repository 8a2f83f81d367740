// Internal structures shared by the host code and the HIP kernels of the
// symed library.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "learned_dev.h"
#include "symed.h"

namespace symed {

constexpr int kMaxSites = 63;

// A flipped pair of sites.  Exchange pieces of every bond on the pair and
// chirality pieces of every triangle edge on the pair flip the same two
// spins, so they merge into one amplitude (J/2 real part, chirality
// imaginary part).
struct PairTerm {
    uint64_t mask;      // both site bits
    uint64_t lo_bit;    // bit of the lower-labelled site
    double Jsum;        // sum of bond couplings on the pair (S^z S^z: Jsum/4 * (+-1))
    int32_t chi_begin;  // range in the chirality-contribution list
    int32_t chi_end;
};

// Contribution of one oriented triangle to the flip of one of its edges:
// Im(h) += c * sgn(site) * sgn_lo, with sgn(site) = +1 if that third spin is
// up, -1 otherwise, and sgn_lo = +1 if the lower-labelled spin of the pair is
// down, -1 otherwise.  (Derivation: S_a.(S_b x S_c) restricted to the flip of
// (b,c) equals (i/2) S^z_a (S^+_b S^-_c - S^-_b S^+_c).)
struct ChiTerm {
    uint64_t site_bit;
    double c;
};

// One move of an SU(d) permutation term on configurations with two bits
// per site (site i's color in the digit at bit offset 2 (n - 1 - i)):
//   kind 0: exchange of the colors of sites (0, 1), <t|H|s> = amp (J);
//   kind 1: cyclic move of three colors, site 0 -> 1 -> 2 -> 0, <t|H|s> = +i amp;
//   kind 2: the inverse cyclic move, <t|H|s> = -i amp
// (a ring term i K (P_ijk - P_ijk^-1) contributes one move of kind 1 and one
// of kind 2 with amp = K).  A move that leaves s unchanged contributes amp
// to the diagonal (kind 0) or nothing (kinds 1 and 2 cancel).
struct ColorMove {
    uint8_t sh[3];   // bit offsets of the three (kind 0: two) digits
    uint8_t kind;
    uint32_t pad;
    double amp;
};

// Everything the kernels need, built on the host.
struct HostTables {
    int N = 0, n_up = 0;
    int G = 0;                          // group order (with flip elements)
    int n_sp = 0;                       // distinct site permutations
    bool has_flip = false;
    bool is_complex = false;
    std::vector<int32_t> sp_of;         // [G]
    std::vector<uint8_t> flip;          // [G]
    std::vector<double> chi_re, chi_im; // [G]
    std::vector<uint8_t> chi_one;       // [G]
    std::vector<int32_t> sp_perm;       // [n_sp][N]

    // Rep/Sym tables on R coarse sublattices of br bits; too large for LDS
    // (rep_global), they stay in device memory and are read through the caches
    int R = 0, br = 0;
    bool rep_global = false;
    std::vector<uint16_t> rep;          // [R][2^br]
    std::vector<uint32_t> sym_off;      // [R*2^br + 1]
    std::vector<uint32_t> sym_list;     // (g << 16) | (sp << 1) | flip
    // SymmetryAction tables on A fine sublattices of ba bits, destination-major.
    // The table of (symmetry, destination d) maps the substate of the source
    // sublattice to the substate it becomes at d; it only depends on how the
    // symmetry orders the sites, so many coincide and each distinct table is
    // stored once.
    int A = 0, ba = 0;
    std::vector<uint16_t> act_tab;      // [n_tab][2^ba]: distinct tables
    std::vector<uint16_t> act_ent;      // [n_sp][A]: (table << 4) | source sublattice

    std::vector<PairTerm> pairs;
    std::vector<ChiTerm> chis;

    // SU(d) permutation models (n_colors > 0): N = 2 * n_sites bits, the group
    // acts on digit pairs; sector = color counts; terms are moves, no pairs
    int n_colors = 0, n_sites = 0;
    int counts[4] = {0, 0, 0, 0};
    std::vector<ColorMove> moves;
};

// Rep/Sym tables: at most this many bytes go to LDS; larger ones stay in
// device memory (up to the second limit; the automatic choice takes at most
// the third, which the L2 cache of one XCD holds twice).
constexpr size_t kRepSymLdsMax = 64 * 1024;
constexpr size_t kRepSymGlobalMax = 16u << 20;
constexpr size_t kRepSymChooseMax = 2u << 20;

// Byte layout of the table blob staged into LDS by the kernels.
struct BlobLayout {
    uint32_t off_rent, off_symlist, off_atab, off_aent, off_pairs, off_chis, off_chi, off_sqrt, off_isqrt, off_chione,
        off_mlp;
    uint32_t aent_lg;    // log2 of the row stride (entries) of the SymmetryAction entries
    // Rep/Sym tables in a separate device buffer (rep_global != 0): their
    // offsets there and its size; off_rent/off_symlist are unused
    uint32_t rep_global, g_rent, g_symlist, gbytes;
    uint32_t off_rank;   // learned index: equalizer, then rank table (after the network pieces; 0 until trained)
    uint32_t off_moves;  // SU(d) models: the ColorMove list
    uint32_t bytes;      // staged into LDS: up to the network pieces and rank table in use
    uint32_t reserved;   // allocated: room for the largest network expansion and rank table
};


// Parameters passed by value to the apply / enumeration kernels.
struct KParams {
    int N, R, br, A, ba, n_pairs, G, is_complex;
    int pbits, n_up;
    int n_colors, n_moves;   // SU(d) models: colors and moves (0 for spin-1/2 models)
    uint64_t maskN;
    BlobLayout lay;
    const void *blob;          // device copy of the LDS blob (16-byte aligned)
    const uint64_t *reps;      // [dim]
    const uint16_t *stab;      // [dim]
    const uint32_t *limits;    // [2^pbits + 1]
    int64_t dim;
    // learned index: the network (expanded) and the rank table live in the
    // LDS blob at lay.off_mlp and lay.off_rank; segments and cells here
    LearnedView lv;
    int32_t has_index;
    // hashed staging table: records {rep, x} (real) or {rep, re, im, -}
    // (complex) in hslots slots, linear probing (null until built)
    const uint64_t *htab;
    uint64_t hslots;
    // learned lookup: {rep, x} records in basis order, one per representative
    // (real sectors; null until the index is trained)
    const uint64_t *lrec;
    // Rep/Sym tables when they live in device memory (lay.rep_global)
    const void *gtab;
};

// Thread-local error reporting.
void set_error(const std::string &msg);
ed_status fail(ed_status st, const std::string &msg);

// tables.cpp
ed_status build_host_tables(const ed_model *m, const ed_group *g, int n_up, int n_sub_rep, int n_sub_act,
                            HostTables &T);
ed_status validate_and_copy_group(const ed_model *m, const ed_group *g, int n_up, HostTables &T);
ed_status check_stable(const HostTables &T, int n_sub);
ed_status check_invariant(const ed_model *m, const HostTables &T);
void build_rep_sym(const HostTables &T, int n_sub, std::vector<uint16_t> &rep, std::vector<uint32_t> &sym_off,
                   std::vector<uint32_t> &sym_list);
void build_pairs(const ed_model *m, HostTables &T);
// LDS blob; with T.rep_global the Rep/Sym tables go to *gblob instead (if
// given; their offsets are set in lay either way).
std::vector<uint8_t> pack_blob(const HostTables &T, BlobLayout &lay, std::vector<uint8_t> *gblob = nullptr);
int choose_sublattices(const HostTables &T, int &R, int &A, std::string &why);
// SU(d) permutation model with colors counts[0..n_colors) (tables.cpp)
ed_status build_color_tables(const ed_model *m, const ed_group *g, int n_colors, const int32_t *counts, int n_sub_rep,
                             int n_sub_act, HostTables &T);

// pwexpand.cpp
int expand_network(const float *params, float mu, float sc, std::vector<float> &block, double *max_dev);

}  // namespace symed
