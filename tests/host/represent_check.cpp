// CPU check of the device representative search (represent.h, compiled for
// the host) against brute force over the whole group, for every state of a
// small instance, or for `samples` random states with n_up spins up
// (SplitMix64 from `seed`, partial Fisher-Yates over the sites) when the
// optional fourth and fifth arguments are given.  Built and run by
// tests/test_represent_host.py.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include "represent.h"
using namespace symed;
template <class T> std::vector<T> rd(FILE *f, size_t n) { std::vector<T> v(n); if (n) fread(v.data(), sizeof(T), n, f); return v; }
int main(int argc, char **argv) {
  FILE *f = fopen(argv[1], "rb"); int R = atoi(argv[2]), A = atoi(argv[3]);
  int32_t hdr[5]; fread(hdr, 4, 5, f);
  int N = hdr[0], n_up = hdr[1], G = hdr[2], nb = hdr[3], nt = hdr[4];
  auto perm = rd<int32_t>(f, (size_t)G * N); auto flip = rd<uint8_t>(f, G);
  auto cre = rd<double>(f, G); auto cim = rd<double>(f, G);
  auto bonds = rd<int32_t>(f, 2 * nb); auto bJ = rd<double>(f, nb);
  auto tris = rd<int32_t>(f, 3 * nt); auto tJ = rd<double>(f, nt);
  fclose(f);
  ed_model m{N, nb, bonds.data(), bJ.data(), nt, tris.data(), tJ.data()};
  ed_group g{G, perm.data(), flip.data(), cre.data(), cim.data()};
  HostTables T;
  ed_status st = build_host_tables(&m, &g, n_up, R, A, T);
  if (st != ED_OK) { printf("build_host_tables failed %d\n", st); return 2; }
  BlobLayout lay; std::vector<uint8_t> gblob; std::vector<uint8_t> blob = pack_blob(T, lay, &gblob);
  std::vector<uint8_t> al(blob.size() + 16); std::memcpy(al.data(), blob.data(), blob.size());
  std::vector<uint8_t> gl(gblob.size() + 16); if (!gblob.empty()) std::memcpy(gl.data(), gblob.data(), gblob.size());
  Lds L = lds_view(al.data(), lay, gl.data());
  // find_rep reports a symmetry by its code (sp << 1) | flip
  std::vector<int> g_of_code(2 * T.n_sp, 0);
  for (int e = 0; e < T.G; ++e) g_of_code[(T.sp_of[e] << 1) | T.flip[e]] = e;
  KParams p{}; p.N = N; p.R = T.R; p.br = T.br; p.A = T.A; p.ba = T.ba; p.maskN = (1ull << N) - 1;
  long long checked = 0, bad = 0;
  const long long samples = argc > 4 ? atoll(argv[4]) : 0;
  uint64_t rng = argc > 5 ? strtoull(argv[5], nullptr, 10) : 1;
  auto next = [&rng]() {
    uint64_t z = (rng += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const uint64_t total = samples ? (uint64_t)samples : (N < 64 ? (1ull << N) : 0);
  for (uint64_t it = 0; it < total; ++it) {
    uint64_t s = it;
    if (samples) {
      int site[64];
      for (int i = 0; i < N; ++i) site[i] = i;
      s = 0;
      for (int k = 0; k < n_up; ++k) {
        int j = k + (int)(next() % (uint64_t)(N - k));
        int t = site[k]; site[k] = site[j]; site[j] = t;
        s |= 1ull << (N - 1 - site[k]);
      }
    } else if (__builtin_popcountll(s) != n_up) {
      continue;
    }
    uint64_t best = ~0ull; int cnt = 0;
    std::vector<uint64_t> img(G);
    for (int e = 0; e < G; ++e) {
      uint64_t o = 0;
      for (int i = 0; i < N; ++i) if ((s >> (N - 1 - i)) & 1) o |= 1ull << (N - 1 - perm[(size_t)e * N + i]);
      if (flip[e]) o ^= p.maskN;
      img[e] = o;
      if (o < best) { best = o; cnt = 1; } else if (o == best) ++cnt;
    }
    Found fr = find_rep(s, p, L);
    ++checked;
    if (fr.rep != best || (int)fr.cnt != cnt || img[g_of_code[fr.g]] != best) {
      if (bad < 5) printf("mismatch s=%llx rep %llx/%llx cnt %u/%d g %u\n", (unsigned long long)s, (unsigned long long)fr.rep, (unsigned long long)best, fr.cnt, cnt, fr.g);
      ++bad;
    }
  }
  printf("R=%d A=%d checked %lld bad %lld\n", T.R, T.A, checked, bad);
  return bad ? 1 : 0;
}
