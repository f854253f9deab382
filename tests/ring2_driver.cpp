// Host-side driver for the test of the L^2 row tables (tests/test_ring2_tables.py):
// reads n, K and the self-padded ELL neighbour table, runs cr::ring2_tables and
// writes the two flags and whichever tables were built.
#include <cstdio>
#include <vector>

#include "ring2.hpp"

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t n = 0;
  int32_t K = 0;
  if (std::fread(&n, 8, 1, f) != 1 || std::fread(&K, 4, 1, f) != 1) return 2;
  std::vector<int32_t> nbr((size_t)K * (size_t)n);
  if (std::fread(nbr.data(), 4, nbr.size(), f) != nbr.size()) return 2;
  std::fclose(f);
  const cr::Ring2Host h = cr::ring2_tables(n, K, nbr.data(), true);
  f = std::fopen(argv[2], "wb");
  if (!f) return 2;
  const int32_t flags[2] = {h.rows ? 1 : 0, h.windows ? 1 : 0};
  std::fwrite(flags, 4, 2, f);
  std::fwrite(h.r2idx.data(), 4, h.r2idx.size(), f);
  std::fwrite(h.r2cf.data(), 1, h.r2cf.size(), f);
  std::fwrite(h.w2tab.data(), 4, h.w2tab.size(), f);
  std::fwrite(h.w2ent.data(), 4, h.w2ent.size(), f);
  std::fclose(f);
  return 0;
}
