// Host side of the symed library: input validation and the lookup tables of
// the sublattice coding technique (thesis, section "Sublattice coding
// techniques": definitions of sublattice stability, G_X, Rep_X, Sym_X and
// SymmetryAction_X; algorithm "Preparation of lookup tables").
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "internal.h"

namespace symed {

namespace {

struct VecHash {
    size_t operator()(const std::vector<int32_t> &v) const {
        size_t h = 1469598103934665603ull;
        for (int32_t x : v) h = (h ^ (uint32_t)x) * 1099511628211ull;
        return h;
    }
};


}  // namespace

// Invariance of an operator under the spatial symmetries: its bonds
// (unordered pairs with summed J) and oriented triangles (sorted triple with
// the sign of the orientation) map onto themselves.  The spin flip is a
// rotation by pi about x, under which both S.S and S.(SxS) are invariant.
ed_status check_invariant(const ed_model *m, const HostTables &T)
{
    const int N = T.N;
    std::map<std::pair<int, int>, double> bonds;
    for (int b = 0; b < m->n_bonds; ++b) {
        int i = m->bond_sites[2 * b], j = m->bond_sites[2 * b + 1];
        bonds[{std::min(i, j), std::max(i, j)}] += m->bond_J[b];
    }
    auto canon_tri = [](int i, int j, int k, double J, std::map<std::array<int, 3>, double> &out) {
        std::array<int, 3> v{i, j, k};
        int sign = 1;
        // bubble sort counting transpositions
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 2 - p; ++q)
                if (v[q] > v[q + 1]) { std::swap(v[q], v[q + 1]); sign = -sign; }
        out[v] += sign * J;
    };
    std::map<std::array<int, 3>, double> tris;
    for (int t = 0; t < m->n_tri; ++t) {
        const int32_t *v = m->tri_sites + 3 * t;
        canon_tri(v[0], v[1], v[2], m->tri_Jchi[t], tris);
    }
    for (int sp = 0; sp < T.n_sp; ++sp) {
        const int32_t *p = &T.sp_perm[(size_t)sp * N];
        std::map<std::pair<int, int>, double> img;
        for (auto &kv : bonds) {
            int i = p[kv.first.first], j = p[kv.first.second];
            img[{std::min(i, j), std::max(i, j)}] += kv.second;
        }
        for (auto &kv : bonds) {
            auto it = img.find(kv.first);
            if (it == img.end() || std::fabs(it->second - kv.second) > 1e-12)
                return fail(ED_EINVAL, "operator (bonds) not invariant under the group");
        }
        std::map<std::array<int, 3>, double> timg;
        for (auto &kv : tris) canon_tri(p[kv.first[0]], p[kv.first[1]], p[kv.first[2]], kv.second, timg);
        for (auto &kv : tris) {
            auto it = timg.find(kv.first);
            double v = (it == timg.end()) ? 0.0 : it->second;
            if (std::fabs(v - kv.second) > 1e-12)
                return fail(ED_EINVAL, "operator (chirality) not invariant under the group");
        }
    }
    return ED_OK;
}

ed_status validate_and_copy_group(const ed_model *m, const ed_group *grp, int n_up, HostTables &T)
{
    if (!m || !grp) return fail(ED_EINVAL, "model and group must not be NULL");
    const int N = m->n_sites;
    if (N < 1 || N > kMaxSites) return fail(ED_EINVAL, "n_sites must be in [1, 63]");
    if (n_up < 0 || n_up > N) return fail(ED_EINVAL, "n_up must be in [0, n_sites]");
    const int G = grp->n_elem;
    if (G < 1 || G > 65535) return fail(ED_EINVAL, "group order must be in [1, 65535]");
    if (!grp->perm || !grp->flip || !grp->chi_re) return fail(ED_EINVAL, "group arrays must not be NULL");
    if (m->n_bonds < 0 || m->n_tri < 0) return fail(ED_EINVAL, "negative term count");
    if (m->n_bonds > 0 && (!m->bond_sites || !m->bond_J)) return fail(ED_EINVAL, "bond arrays NULL");
    if (m->n_tri > 0 && (!m->tri_sites || !m->tri_Jchi)) return fail(ED_EINVAL, "triangle arrays NULL");
    for (int b = 0; b < m->n_bonds; ++b) {
        int i = m->bond_sites[2 * b], j = m->bond_sites[2 * b + 1];
        if (i < 0 || i >= N || j < 0 || j >= N || i == j) return fail(ED_EINVAL, "bad bond " + std::to_string(b));
        if (!std::isfinite(m->bond_J[b])) return fail(ED_EINVAL, "non-finite bond coupling");
    }
    for (int t = 0; t < m->n_tri; ++t) {
        const int32_t *v = m->tri_sites + 3 * t;
        for (int q = 0; q < 3; ++q)
            if (v[q] < 0 || v[q] >= N) return fail(ED_EINVAL, "bad triangle " + std::to_string(t));
        if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) return fail(ED_EINVAL, "degenerate triangle");
        if (!std::isfinite(m->tri_Jchi[t])) return fail(ED_EINVAL, "non-finite chirality coupling");
    }

    T = HostTables();
    T.N = N;
    T.n_up = n_up;
    T.G = G;
    T.sp_of.resize(G);
    T.flip.resize(G);
    T.chi_re.resize(G);
    T.chi_im.resize(G);
    T.chi_one.resize(G);

    std::unordered_map<std::vector<int32_t>, int, VecHash> sp_index;
    std::vector<int32_t> perm(N);
    for (int g = 0; g < G; ++g) {
        std::vector<uint8_t> seen(N, 0);
        for (int i = 0; i < N; ++i) {
            int32_t j = grp->perm[(size_t)g * N + i];
            if (j < 0 || j >= N || seen[j]) return fail(ED_EINVAL, "group element " + std::to_string(g) + " is not a permutation");
            seen[j] = 1;
            perm[i] = j;
        }
        auto it = sp_index.find(perm);
        int sp;
        if (it == sp_index.end()) {
            sp = T.n_sp++;
            sp_index.emplace(perm, sp);
            T.sp_perm.insert(T.sp_perm.end(), perm.begin(), perm.end());
        } else {
            sp = it->second;
        }
        T.sp_of[g] = sp;
        T.flip[g] = grp->flip[g] ? 1 : 0;
        T.chi_re[g] = grp->chi_re[g];
        T.chi_im[g] = grp->chi_im ? grp->chi_im[g] : 0.0;
        double mod = std::hypot(T.chi_re[g], T.chi_im[g]);
        if (!(std::fabs(mod - 1.0) < 1e-9)) return fail(ED_ECHAR, "|chi| != 1 at element " + std::to_string(g));
        T.chi_one[g] = std::hypot(T.chi_re[g] - 1.0, T.chi_im[g]) < 1e-6 ? 1 : 0;
        if (T.flip[g]) T.has_flip = true;
    }
    if (T.has_flip && 2 * n_up != N) return fail(ED_EINVAL, "spin flip requires n_up == n_sites/2");
    if (T.n_sp > 32767) return fail(ED_EINVAL, "too many distinct permutations");

    // closure and multiplicativity: (g h) = perm_g o perm_h, flip_g ^ flip_h
    std::unordered_map<long long, int> elem;   // key: sp * 2 + flip
    for (int g = 0; g < G; ++g) {
        long long key = (long long)T.sp_of[g] * 2 + T.flip[g];
        if (elem.count(key)) return fail(ED_EINVAL, "duplicate group element " + std::to_string(g));
        elem[key] = g;
    }
    std::vector<int32_t> comp(N);
    for (int a = 0; a < G; ++a) {
        const int32_t *pa = &T.sp_perm[(size_t)T.sp_of[a] * N];
        for (int b = 0; b < G; ++b) {
            const int32_t *pb = &T.sp_perm[(size_t)T.sp_of[b] * N];
            for (int i = 0; i < N; ++i) comp[i] = pa[pb[i]];
            auto it = sp_index.find(comp);
            if (it == sp_index.end()) return fail(ED_EINVAL, "group not closed under composition");
            auto e = elem.find((long long)it->second * 2 + (T.flip[a] ^ T.flip[b]));
            if (e == elem.end()) return fail(ED_EINVAL, "group not closed under composition");
            int c = e->second;
            double re = T.chi_re[a] * T.chi_re[b] - T.chi_im[a] * T.chi_im[b];
            double im = T.chi_re[a] * T.chi_im[b] + T.chi_im[a] * T.chi_re[b];
            if (std::hypot(re - T.chi_re[c], im - T.chi_im[c]) > 1e-9)
                return fail(ED_ECHAR, "characters are not multiplicative");
        }
    }

    ed_status inv = check_invariant(m, T);
    if (inv != ED_OK) return inv;
    bool cplx_chi = false;
    for (int g = 0; g < G; ++g)
        if (std::fabs(T.chi_im[g]) > 1e-12) cplx_chi = true;
    bool has_chir = false;
    for (int t = 0; t < m->n_tri; ++t)
        if (m->tri_Jchi[t] != 0.0) has_chir = true;
    T.is_complex = cplx_chi || has_chir;
    return ED_OK;
}

ed_status check_stable(const HostTables &T, int n_sub)
{
    if (n_sub < 1 || T.N % n_sub) return fail(ED_ENOTSTABLE, "n_sites not divisible by the number of sublattices");
    int b = T.N / n_sub;
    for (int sp = 0; sp < T.n_sp; ++sp) {
        const int32_t *p = &T.sp_perm[(size_t)sp * T.N];
        for (int X = 0; X < n_sub; ++X) {
            int Y = p[X * b] / b;
            for (int q = 1; q < b; ++q)
                if (p[X * b + q] / b != Y)
                    return fail(ED_ENOTSTABLE, "sublattice decomposition into " + std::to_string(n_sub) +
                                                   " contiguous blocks is not stable under the group");
        }
    }
    return ED_OK;
}

// image of the b-bit substate s of block X under spatial permutation p, as a
// b-bit substate of the destination block (bits in within-block order)
static inline uint32_t sub_image(const int32_t *p, int X, int b, uint32_t s)
{
    uint32_t out = 0;
    for (int q = 0; q < b; ++q)
        if ((s >> (b - 1 - q)) & 1u) {
            int j = p[X * b + q];
            out |= 1u << (b - 1 - (j % b));
        }
    return out;
}

void build_rep_sym(const HostTables &T, int n_sub, std::vector<uint16_t> &rep, std::vector<uint32_t> &sym_off,
                   std::vector<uint32_t> &sym_list)
{
    const int b = T.N / n_sub;
    const uint32_t S = 1u << b, mask = S - 1;
    rep.assign((size_t)n_sub * S, 0);
    sym_off.assign((size_t)n_sub * S + 1, 0);
    sym_list.clear();
    // G_X: elements mapping sublattice X onto sublattice 0 (definition of
    // the sublattice symmetries)
    std::vector<std::vector<int>> GX(n_sub);
    for (int g = 0; g < T.G; ++g) {
        const int32_t *p = &T.sp_perm[(size_t)T.sp_of[g] * T.N];
        for (int X = 0; X < n_sub; ++X)
            if (p[X * b] / b == 0) GX[X].push_back(g);
    }
    // The image of a substate is the OR of the images of its bits, so it is
    // assembled from the images of its 8-bit chunks (one table per element;
    // every caller keeps b <= 16, so at most two chunks).
    const int nc = (b + 7) / 8;
    std::vector<uint32_t> chunk, best;
    for (int X = 0; X < n_sub; ++X) {
        const size_t ng = GX[X].size();
        chunk.assign(ng * nc * 256, 0u);
        for (size_t k = 0; k < ng; ++k) {
            const int32_t *p = &T.sp_perm[(size_t)T.sp_of[GX[X][k]] * T.N];
            for (int c = 0; c < nc; ++c)
                for (uint32_t u = 0; u < 256; ++u)
                    chunk[(k * nc + c) * 256 + u] = sub_image(p, X, b, (u << (8 * c)) & mask);
        }
        std::vector<uint32_t> fm(ng);
        for (size_t k = 0; k < ng; ++k) fm[k] = T.flip[GX[X][k]] ? mask : 0u;
        auto image = [&](size_t k, uint32_t s) {
            const uint32_t *t = chunk.data() + k * nc * 256;
            uint32_t v = t[s & 255u];
            if (nc > 1) v |= t[256 + ((s >> 8) & 255u)];
            return v ^ fm[k];
        };
        best.assign(S, ~0u);
        for (size_t k = 0; k < ng; ++k)
            for (uint32_t s = 0; s < S; ++s) best[s] = std::min(best[s], image(k, s));
        for (uint32_t s = 0; s < S; ++s) {
            rep[(size_t)X * S + s] = (uint16_t)best[s];
            for (size_t k = 0; k < ng; ++k)
                if (image(k, s) == best[s]) {
                    int g = GX[X][k];
                    sym_list.push_back(((uint32_t)g << 16) | ((uint32_t)T.sp_of[g] << 1) | T.flip[g]);
                }
            sym_off[(size_t)X * S + s + 1] = (uint32_t)sym_list.size();
        }
    }
}

// Distinct SymmetryAction tables of the decomposition into A sublattices
// (at most `limit`; -1 if there are more).  rows / tabs receive them if given.
static int act_tables(const HostTables &T, int A, int limit, std::vector<uint16_t> *ents, std::vector<uint16_t> *tabs)
{
    const int b = T.N / A;
    const uint32_t S = 1u << b;
    // the map from source positions to destination positions identifies a table
    std::map<std::vector<uint8_t>, int> ids;
    if (ents) ents->assign((size_t)T.n_sp * A, 0);
    if (tabs) tabs->clear();
    std::vector<uint8_t> key(b);
    for (int sp = 0; sp < T.n_sp; ++sp) {
        const int32_t *p = &T.sp_perm[(size_t)sp * T.N];
        for (int X = 0; X < A; ++X) {
            const int d = p[X * b] / b;  // destination of X
            for (int q = 0; q < b; ++q) key[q] = (uint8_t)(p[X * b + q] % b);
            auto it = ids.find(key);
            int id;
            if (it == ids.end()) {
                id = (int)ids.size();
                if (id >= limit) return -1;
                ids.emplace(key, id);
                if (tabs)
                    for (uint32_t s = 0; s < S; ++s) tabs->push_back((uint16_t)sub_image(p, X, b, s));
            } else {
                id = it->second;
            }
            if (ents) (*ents)[(size_t)sp * A + d] = (uint16_t)((id << 4) | X);
        }
    }
    return (int)ids.size();
}

static ed_status build_act(HostTables &T)
{
    if (act_tables(T, T.A, 4096, &T.act_ent, &T.act_tab) < 0)
        return fail(ED_EINVAL, "more than 4096 distinct SymmetryAction tables; choose more sublattices");
    return ED_OK;
}

void build_pairs(const ed_model *m, HostTables &T)
{
    const int N = T.N;
    std::map<std::pair<int, int>, double> J;
    std::map<std::pair<int, int>, std::vector<ChiTerm>> C;
    for (int b = 0; b < m->n_bonds; ++b) {
        int i = m->bond_sites[2 * b], j = m->bond_sites[2 * b + 1];
        J[{std::min(i, j), std::max(i, j)}] += m->bond_J[b];
    }
    for (int t = 0; t < m->n_tri; ++t) {
        const int32_t *v = m->tri_sites + 3 * t;
        double Jc = m->tri_Jchi[t];
        if (Jc == 0.0) continue;
        for (int r = 0; r < 3; ++r) {
            int a = v[r], bb = v[(r + 1) % 3], c = v[(r + 2) % 3];
            int lo = std::min(bb, c), hi = std::max(bb, c);
            double o = (bb == lo) ? 1.0 : -1.0;
            C[{lo, hi}].push_back(ChiTerm{(uint64_t)1 << (N - 1 - a), o * Jc / 4.0});
            J[{lo, hi}] += 0.0;
        }
    }
    T.pairs.clear();
    T.chis.clear();
    for (auto &kv : J) {
        PairTerm pt;
        int lo = kv.first.first, hi = kv.first.second;
        pt.lo_bit = (uint64_t)1 << (N - 1 - lo);
        pt.mask = pt.lo_bit | ((uint64_t)1 << (N - 1 - hi));
        pt.Jsum = kv.second;
        pt.chi_begin = (int32_t)T.chis.size();
        auto it = C.find(kv.first);
        if (it != C.end())
            for (auto &ct : it->second) T.chis.push_back(ct);
        pt.chi_end = (int32_t)T.chis.size();
        T.pairs.push_back(pt);
    }
}

static size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

std::vector<uint8_t> pack_blob(const HostTables &T, BlobLayout &L, std::vector<uint8_t> *gblob)
{
    // Rep/Sym entries {Rep | count << 16, first Sym entry} (8 B per substate)
    // and SymList u16 (symmetry codes): in the LDS blob, or in a buffer of
    // their own
    size_t o = 0, g = 0;
    size_t &rs = T.rep_global ? g : o;
    L.rep_global = T.rep_global ? 1u : 0u;
    const uint32_t r0 = (uint32_t)rs;    rs = align16(rs + T.rep.size() * 2 * sizeof(uint32_t));
    const uint32_t r1 = (uint32_t)rs;    rs = align16(rs + T.sym_list.size() * sizeof(uint16_t));
    L.off_rent = L.off_symlist = 0;
    L.g_rent = L.g_symlist = 0;
    if (T.rep_global) {
        L.g_rent = r0;
        L.g_symlist = r1;
    } else {
        L.off_rent = r0;
        L.off_symlist = r1;
    }
    L.gbytes = (uint32_t)g;
    L.off_atab = (uint32_t)o;    o = align16(o + T.act_tab.size() * sizeof(uint16_t));
    // entry rows padded to a power-of-two stride (a shift instead of a multiply)
    L.aent_lg = 0;
    while ((1 << L.aent_lg) < T.A) ++L.aent_lg;
    L.off_aent = (uint32_t)o;    o = align16(o + ((size_t)T.n_sp << L.aent_lg) * sizeof(uint32_t));
    L.off_pairs = (uint32_t)o;   o = align16(o + T.pairs.size() * sizeof(PairTerm));
    L.off_chis = (uint32_t)o;    o = align16(o + T.chis.size() * sizeof(ChiTerm));
    L.off_moves = (uint32_t)o;   o = align16(o + T.moves.size() * sizeof(ColorMove));
    L.off_chi = (uint32_t)o;     o = align16(o + (size_t)2 * T.n_sp * sizeof(double) * (T.is_complex ? 2 : 1));
    L.off_sqrt = (uint32_t)o;    o = align16(o + (size_t)(T.G + 1) * sizeof(double));
    L.off_isqrt = (uint32_t)o;   o = align16(o + (size_t)(T.G + 1) * sizeof(double));
    L.off_chione = (uint32_t)o;  o = align16(o + (size_t)2 * T.n_sp);
    // space for the learned index, filled after training: the network in
    // expanded form, then the equalizer and the rank table right behind the
    // pieces in use
    L.off_mlp = (uint32_t)o;
    L.off_rank = 0;
    L.bytes = (uint32_t)align16(o + kPwHeader * sizeof(float));   // no network yet: header only
    o = o + (size_t)kLearnedLdsMax;
    L.reserved = (uint32_t)o;
    std::vector<uint8_t> blob(o, 0);
    auto put = [&](uint32_t off, const void *src, size_t n) { if (n) std::memcpy(blob.data() + off, src, n); };
    // device form of the Sym list: for each symmetry its code (sp << 1) | flip;
    // counts fit 16 bits since the group has at most 65535 elements
    std::vector<uint16_t> code(T.sym_list.size());
    for (size_t k = 0; k < T.sym_list.size(); ++k) code[k] = (uint16_t)(T.sym_list[k] & 0xffffu);
    std::vector<uint32_t> rent(2 * T.rep.size());
    for (size_t i = 0; i < T.rep.size(); ++i) {
        rent[2 * i] = (uint32_t)T.rep[i] | ((T.sym_off[i + 1] - T.sym_off[i]) << 16);
        rent[2 * i + 1] = T.sym_off[i];
    }
    if (!T.rep_global) {
        put(L.off_rent, rent.data(), rent.size() * sizeof(uint32_t));
        put(L.off_symlist, code.data(), code.size() * sizeof(uint16_t));
    } else if (gblob) {
        gblob->assign(g, 0);
        auto gput = [&](uint32_t off, const void *src, size_t n) { if (n) std::memcpy(gblob->data() + off, src, n); };
        gput(L.g_rent, rent.data(), rent.size() * sizeof(uint32_t));
        gput(L.g_symlist, code.data(), code.size() * sizeof(uint16_t));
    }
    put(L.off_atab, T.act_tab.data(), T.act_tab.size() * sizeof(uint16_t));
    // device form of the entries: byte offset of the table in atab << 8 |
    // right shift of the source substate (byte offsets < 2^24: the blob
    // fits LDS; shifts < 64)
    std::vector<uint32_t> ent32((size_t)T.n_sp << L.aent_lg, 0u);
    for (int sp = 0; sp < T.n_sp; ++sp)
        for (int d = 0; d < T.A; ++d) {
            const uint32_t e = T.act_ent[(size_t)sp * T.A + d], X = e & 15u;
            const uint32_t byte_off = ((e >> 4) << T.ba) * (uint32_t)sizeof(uint16_t);
            ent32[((size_t)sp << L.aent_lg) + d] = (byte_off << 8) | (uint32_t)(T.N - (int)(X + 1) * T.ba);
        }
    put(L.off_aent, ent32.data(), ent32.size() * sizeof(uint32_t));
    put(L.off_pairs, T.pairs.data(), T.pairs.size() * sizeof(PairTerm));
    put(L.off_chis, T.chis.data(), T.chis.size() * sizeof(ChiTerm));
    put(L.off_moves, T.moves.data(), T.moves.size() * sizeof(ColorMove));
    // characters and the "chi == 1" flags by symmetry code (sp << 1) | flip
    const int w = T.is_complex ? 2 : 1;
    std::vector<double> chi((size_t)2 * T.n_sp * w, 0.0);
    std::vector<uint8_t> one((size_t)2 * T.n_sp, 0);
    for (int g = 0; g < T.G; ++g) {
        const size_t c = ((size_t)T.sp_of[g] << 1) | T.flip[g];
        chi[c * w] = T.chi_re[g];
        if (T.is_complex) chi[c * w + 1] = T.chi_im[g];
        one[c] = T.chi_one[g];
    }
    put(L.off_chi, chi.data(), chi.size() * sizeof(double));
    std::vector<double> sq(T.G + 1), isq(T.G + 1);
    for (int k = 0; k <= T.G; ++k) {
        sq[k] = std::sqrt((double)k);
        isq[k] = k ? 1.0 / std::sqrt((double)k) : 0.0;
    }
    put(L.off_sqrt, sq.data(), sq.size() * sizeof(double));
    put(L.off_isqrt, isq.data(), isq.size() * sizeof(double));
    put(L.off_chione, one.data(), one.size());
    return blob;
}

// Bytes of the device Rep/Sym tables: an 8 B entry per substate (Rep,
// number of Sym entries, first Sym entry) and a u16 code per Sym entry.
static size_t rep_sym_bytes(size_t n_rep, size_t n_list) { return n_rep * 8 + n_list * 2; }

// Choose the decompositions: the SymmetryAction tables use the stable
// contiguous decomposition with the fewest sublattices (fewest destination
// steps per candidate) whose distinct tables fit (<= 12 bits per substate,
// <= 16 sublattices, tables of <= 48 KiB together); the Rep/Sym
// tables use the one with the fewest sublattices (fewest candidate
// symmetries) that the action decomposition refines and whose tables fit
// 64 KiB of LDS, or 2 MiB of device memory read through the caches.
int choose_sublattices(const HostTables &T, int &R, int &A, std::string &why)
{
    const int N = T.N;
    std::vector<int> stable;
    for (int ns = 1; ns <= N; ++ns) {
        if (N % ns) continue;
        std::string save;
        if (check_stable(T, ns) == ED_OK) stable.push_back(ns);
    }
    set_error("");
    int bestA = 0;
    for (int ns : stable) {
        int b = N / ns;
        if (b > 12 || ns > 16) continue;
        const size_t per = ((size_t)1 << b) * sizeof(uint16_t);
        const int limit = (int)std::min<size_t>(4096, 48 * 1024 / per);
        if (limit < 1 || act_tables(T, ns, limit, nullptr, nullptr) < 0) continue;
        // the Rep/Sym decomposition must divide it: some stable one with small enough tables
        bool refinable = false;
        for (int r : stable)
            if (ns % r == 0 && N / r <= 16) refinable = true;
        if (refinable) { bestA = ns; break; }
    }
    if (!bestA) {
        why = "no stable decomposition gives distinct SymmetryAction tables within 48 KiB";
        return 0;
    }
    int bestR = 0;
    for (int ns : stable) {
        if (bestA % ns) continue;  // the action decomposition must refine this one
        int b = N / ns;
        if (b > 16) continue;
        size_t S = (size_t)1 << b;
        if (rep_sym_bytes(ns * S, 0) > kRepSymChooseMax) continue;
        std::vector<uint16_t> rep;
        std::vector<uint32_t> off, lst;
        build_rep_sym(T, ns, rep, off, lst);
        if (rep_sym_bytes(rep.size(), lst.size()) <= kRepSymChooseMax) { bestR = ns; break; }
    }
    if (!bestR) {
        why = "no stable decomposition gives Rep/Sym tables of at most 2 MiB";
        return 0;
    }
    R = bestR;
    A = bestA;
    return 1;
}

ed_status build_host_tables(const ed_model *m, const ed_group *g, int n_up, int n_sub_rep, int n_sub_act,
                            HostTables &T)
{
    ed_status st = validate_and_copy_group(m, g, n_up, T);
    if (st != ED_OK) return st;
    int R = n_sub_rep, A = n_sub_act;
    if (R <= 0 || A <= 0) {
        int Ra = 0, Aa = 0;
        std::string why;
        if (!choose_sublattices(T, Ra, Aa, why)) return fail(ED_ENOTSTABLE, why);
        if (R <= 0) R = Ra;
        if (A <= 0) A = Aa;
    }
    if ((st = check_stable(T, R)) != ED_OK) return st;
    if ((st = check_stable(T, A)) != ED_OK) return st;
    if (A % R) return fail(ED_EINVAL, "n_sub_act must be a multiple of n_sub_rep");
    T.R = R;
    T.br = T.N / R;
    T.A = A;
    T.ba = T.N / A;
    if (T.br > 16) return fail(ED_EINVAL, "Rep/Sym substates wider than 16 bits");
    if (T.ba > 12 || A > 16)
        return fail(ED_EINVAL, "SymmetryAction tables need <= 12 bits per substate and <= 16 sublattices");
    build_rep_sym(T, R, T.rep, T.sym_off, T.sym_list);
    if (T.n_sp >= 32768) return fail(ED_EINVAL, "too many distinct permutations for 16-bit symmetry codes");
    const size_t rs_bytes = rep_sym_bytes(T.rep.size(), T.sym_list.size());
    if (rs_bytes > kRepSymGlobalMax)
        return fail(ED_EINVAL, "Rep/Sym tables of " + std::to_string(rs_bytes) + " B; choose more Rep sublattices");
    T.rep_global = rs_bytes > kRepSymLdsMax;
    if ((st = build_act(T)) != ED_OK) return st;
    build_pairs(m, T);
    return ED_OK;
}

// SU(d) permutation model H = sum_b J_b P_ij + sum_t K_t i (P_ijk - P_ijk^-1)
// (thesis, chapter on SU(N) chiral spin liquids: the SU(N) Heisenberg model
// with imaginary ring exchange on elementary triangles).  A site holds a
// color 0..d-1 in two bits, so a configuration of n sites is a 2n-bit integer
// (site 0 in the most significant digit) and a site permutation is a
// permutation of bit positions, 2i + t -> 2 perm(i) + t.  The sublattice
// coding tables, the representative search and the index lookups are those
// of the spin-1/2 case on these 2n bit positions; only the sector (color
// counts instead of a number of up spins) and the terms differ.
// The ring term is totally antisymmetric in (i, j, k), like the scalar
// chirality (for d = 2 it equals 4 S_i.(S_j x S_k)), so the invariance check
// of the spin-1/2 model applies to the site-level model unchanged.
ed_status build_color_tables(const ed_model *m, const ed_group *g, int n_colors, const int32_t *counts, int n_sub_rep,
                             int n_sub_act, HostTables &T)
{
    if (!m || !g) return fail(ED_EINVAL, "model and group must not be NULL");
    if (n_colors < 2 || n_colors > 4) return fail(ED_EINVAL, "n_colors must be in [2, 4]");
    if (!counts) return fail(ED_EINVAL, "counts must not be NULL");
    const int n = m->n_sites;
    if (n < 1 || 2 * n > 62) return fail(ED_EINVAL, "n_sites must be in [1, 31] for two bits per site");
    int sum = 0;
    for (int c = 0; c < n_colors; ++c) {
        if (counts[c] < 0) return fail(ED_EINVAL, "negative color count");
        sum += counts[c];
    }
    if (sum != n) return fail(ED_EINVAL, "color counts must add up to n_sites");
    if (g->n_elem >= 1 && g->flip)
        for (int e = 0; e < g->n_elem; ++e)
            if (g->flip[e]) return fail(ED_EINVAL, "spin-flip elements are not defined for SU(d) models");
    // site level: group closure, characters, invariance of the terms
    HostTables S;
    ed_status st = validate_and_copy_group(m, g, 0, S);
    if (st != ED_OK) return st;

    // bit level: the same group acting on the 2n bit positions, no terms
    const int N = 2 * n, G = g->n_elem;
    std::vector<int32_t> bperm((size_t)G * N);
    for (int e = 0; e < G; ++e)
        for (int i = 0; i < n; ++i)
            for (int t = 0; t < 2; ++t) bperm[(size_t)e * N + 2 * i + t] = 2 * g->perm[(size_t)e * n + i] + t;
    std::vector<uint8_t> bflip(G, 0);
    ed_group bg{G, bperm.data(), bflip.data(), g->chi_re, g->chi_im};
    ed_model bm{N, 0, nullptr, nullptr, 0, nullptr, nullptr};
    if ((st = build_host_tables(&bm, &bg, 0, n_sub_rep, n_sub_act, T)) != ED_OK) return st;
    T.n_colors = n_colors;
    T.n_sites = n;
    for (int c = 0; c < 4; ++c) T.counts[c] = c < n_colors ? counts[c] : 0;

    // moves: exchange couplings summed per unordered pair; ring couplings
    // summed per triangle, each taken in the rotation that starts at its
    // smallest site, with the sign of K reversed for the opposite orientation
    std::map<std::pair<int, int>, double> J;
    for (int b = 0; b < m->n_bonds; ++b) {
        const int i = m->bond_sites[2 * b], j = m->bond_sites[2 * b + 1];
        J[{std::min(i, j), std::max(i, j)}] += m->bond_J[b];
    }
    std::map<std::array<int, 3>, double> K;
    for (int t = 0; t < m->n_tri; ++t) {
        const int32_t *v = m->tri_sites + 3 * t;
        int r = 0;
        for (int q = 1; q < 3; ++q)
            if (v[q] < v[r]) r = q;
        const int a = v[r], b = v[(r + 1) % 3], c = v[(r + 2) % 3];
        if (b < c) K[{a, b, c}] += m->tri_Jchi[t];
        else K[{a, c, b}] -= m->tri_Jchi[t];
    }
    auto off = [n](int i) { return (uint8_t)(2 * (n - 1 - i)); };
    T.moves.clear();
    for (auto &kv : J) {
        if (kv.second == 0.0) continue;
        ColorMove mv{};
        mv.sh[0] = off(kv.first.first);
        mv.sh[1] = off(kv.first.second);
        mv.kind = 0;
        mv.amp = kv.second;
        T.moves.push_back(mv);
    }
    bool ring = false;
    for (auto &kv : K) {
        if (kv.second == 0.0) continue;
        ring = true;
        for (uint8_t kind = 1; kind <= 2; ++kind) {
            ColorMove mv{};
            for (int q = 0; q < 3; ++q) mv.sh[q] = off(kv.first[q]);
            mv.kind = kind;
            mv.amp = kv.second;
            T.moves.push_back(mv);
        }
    }
    T.is_complex = T.is_complex || ring;
    return ED_OK;
}

}  // namespace symed
