// CPU check of the SU(d) device code compiled for the host (colors_dev.h,
// represent.h, and build_color_tables from the library's objects):
//  - color_unrank(r) for every rank equals the r-th configuration reached by
//    color_next from 0, and color_next(t) is the smallest sector
//    configuration >= t for random t (brute force over the sector);
//  - find_rep on every sector configuration equals the brute-force minimum
//    over the group (representative, stabilizer size, a reaching element);
//  - the enumeration of the GPU kernel, chunk by chunk with the given chunk
//    length and the same prefix pruning, is written to the output file with
//    each representative's stabilizer and the moves' action on it (target,
//    amplitude) for the Python test to compare with the oracle.
// Input file: int32 n_sites, d, G, n_bonds, n_tri, counts[4], then perm,
// flip, chi_re, chi_im, bonds, bond_J, tris, tri_K.  Built and run by
// tests/test_colors_host.py.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include "colors_dev.h"
using namespace symed;
template <class T> std::vector<T> rd(FILE *f, size_t n) { std::vector<T> v(n); if (n) fread(v.data(), sizeof(T), n, f); return v; }
int main(int argc, char **argv) {
  FILE *f = fopen(argv[1], "rb"); int R = atoi(argv[2]), A = atoi(argv[3]);
  const uint64_t len = strtoull(argv[4], nullptr, 10);
  int32_t hdr[9]; fread(hdr, 4, 9, f);
  int n = hdr[0], d = hdr[1], G = hdr[2], nb = hdr[3], nt = hdr[4];
  int32_t counts[4] = {hdr[5], hdr[6], hdr[7], hdr[8]};
  auto perm = rd<int32_t>(f, (size_t)G * n); auto flip = rd<uint8_t>(f, G);
  auto cre = rd<double>(f, G); auto cim = rd<double>(f, G);
  auto bonds = rd<int32_t>(f, 2 * nb); auto bJ = rd<double>(f, nb);
  auto tris = rd<int32_t>(f, 3 * nt); auto tK = rd<double>(f, nt);
  fclose(f);
  ed_model m{n, nb, bonds.data(), bJ.data(), nt, tris.data(), tK.data()};
  ed_group g{G, perm.data(), flip.data(), cre.data(), cim.data()};
  HostTables T;
  ed_status st = build_color_tables(&m, &g, d, counts, R, A, T);
  if (st != ED_OK) { printf("build_color_tables failed %d\n", st); return 2; }
  BlobLayout lay; std::vector<uint8_t> gblob; std::vector<uint8_t> blob = pack_blob(T, lay, &gblob);
  std::vector<uint8_t> al(blob.size() + 16); std::memcpy(al.data(), blob.data(), blob.size());
  std::vector<uint8_t> gl(gblob.size() + 16); if (!gblob.empty()) std::memcpy(gl.data(), gblob.data(), gblob.size());
  Lds L = lds_view(al.data(), lay, gl.data());
  const int N = T.N;
  KParams p{}; p.N = N; p.R = T.R; p.br = T.br; p.A = T.A; p.ba = T.ba; p.maskN = (1ull << N) - 1;
  p.n_colors = d; p.n_moves = (int)T.moves.size();
  std::vector<int> g_of_code(2 * T.n_sp, 0);
  for (int e = 0; e < T.G; ++e) g_of_code[(T.sp_of[e] << 1) | T.flip[e]] = e;
  ColorSector cs{}; cs.n = n; cs.d = d; for (int c = 0; c < 4; ++c) cs.cnt[c] = counts[c];
  long long bad = 0;
  // the whole sector by color_next, and the ranks
  std::vector<uint64_t> all;
  for (uint64_t s = color_next(0, cs); s != kNoConfig; s = color_next(s + 1, cs)) all.push_back(s);
  const uint64_t total = all.size();
  for (uint64_t r = 0; r < total; ++r)
    if (color_unrank(r, total, cs) != all[r]) { if (bad++ < 5) printf("unrank %llu\n", (unsigned long long)r); }
  // color_next on arbitrary integers below 4^n
  uint64_t rng = 12345;
  for (int it = 0; it < 20000; ++it) {
    rng = rng * 6364136223846793005ull + 1442695040888963407ull;
    const uint64_t t = (rng >> 11) % (p.maskN + 1);
    auto it2 = std::lower_bound(all.begin(), all.end(), t);
    const uint64_t want = it2 == all.end() ? kNoConfig : *it2;
    if (color_next(t, cs) != want) { if (bad++ < 5) printf("next %llx\n", (unsigned long long)t); }
  }
  // representative search against brute force
  for (uint64_t s : all) {
    uint64_t best = ~0ull; int cnt = 0; std::vector<uint64_t> img(G);
    for (int e = 0; e < G; ++e) {
      uint64_t o = 0;
      for (int i = 0; i < n; ++i) o |= ((s >> (2 * (n - 1 - i))) & 3ull) << (2 * (n - 1 - perm[(size_t)e * n + i]));
      img[e] = o;
      if (o < best) { best = o; cnt = 1; } else if (o == best) ++cnt;
    }
    Found fr = find_rep(s, p, L);
    if (fr.rep != best || (int)fr.cnt != cnt || img[g_of_code[fr.g]] != best) {
      if (bad++ < 5) printf("find_rep s=%llx\n", (unsigned long long)s);
    }
  }
  // enumeration as in the kernel: chunks of len ranks, prefix pruning
  std::vector<uint64_t> reps; std::vector<uint32_t> stabs;
  const uint64_t n_chunks = total ? (total + len - 1) / len : 1;
  for (uint64_t c = 0; c < n_chunks; ++c) {
    const uint64_t r0 = c * len, r1 = std::min(total, r0 + len);
    uint64_t s = color_unrank(r0, total, cs);
    const uint64_t send = r1 < total ? color_unrank(r1, total, cs) : kNoConfig;
    while (s < send) {
      const int badX = rep_prefix_fail(s, p, L);
      if (badX >= 0) { const int sh = N - (badX + 1) * p.br; s = color_next(((s >> sh) + 1) << sh, cs); continue; }
      uint32_t stb = 0; bool triv = true;
      if (rep_check(s, p, L, stb, triv) && triv) { reps.push_back(s); stabs.push_back(stb); }
      s = color_next(s + 1, cs);
    }
  }
  FILE *o = fopen(argv[5], "wb");
  const uint64_t dim = reps.size();
  fwrite(&dim, 8, 1, o);
  fwrite(reps.data(), 8, dim, o);
  fwrite(stabs.data(), 4, dim, o);
  // per representative: diagonal, then the moves that change it
  for (uint64_t s : reps) {
    double diag = 0.0; std::vector<uint64_t> tg; std::vector<double> hr, hi;
    for (const ColorMove &mv : T.moves) {
      const uint64_t t = move_target(s, mv);
      if (t == s) { if (mv.kind == 0) diag += mv.amp; continue; }
      double a, b; move_amp(mv, a, b); tg.push_back(t); hr.push_back(a); hi.push_back(b);
    }
    const uint64_t k = tg.size();
    fwrite(&diag, 8, 1, o); fwrite(&k, 8, 1, o);
    fwrite(tg.data(), 8, k, o); fwrite(hr.data(), 8, k, o); fwrite(hi.data(), 8, k, o);
  }
  fclose(o);
  printf("R=%d A=%d total %llu dim %llu complex %d moves %zu bad %lld\n", T.R, T.A, (unsigned long long)total,
         (unsigned long long)dim, T.is_complex ? 1 : 0, T.moves.size(), bad);
  return bad ? 1 : 0;
}
