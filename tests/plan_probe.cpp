// Host-only probe of the library's plan for the CPU tests: reads a topology
// (M, N, K, L, obs_cam[K], obs_pt[K], cam_block[M] as int32) and prints the
// internal camera order, the nonzero-tile flags of every sub-block's factor
// and the length of the dataflow task list (0 = the order check failed).
#include <cstdio>
#include <vector>

#include "rpba_plan.hpp"

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t h[4];
  if (std::fread(h, 4, 4, f) != 4) return 2;
  const int32_t M = h[0], N = h[1], K = h[2], L = h[3];
  std::vector<int32_t> oc(K), op(K), cb(M);
  if (std::fread(oc.data(), 4, K, f) != (size_t)K || std::fread(op.data(), 4, K, f) != (size_t)K ||
      std::fread(cb.data(), 4, M, f) != (size_t)M)
    return 2;
  std::fclose(f);
  rpba::Plan P;
  const std::string e = rpba::build_plan(M, N, K, L, oc.data(), op.data(), cb.data(), 64, 6, P);
  if (!e.empty()) {
    std::printf("error %s\n", e.c_str());
    return 1;
  }
  std::printf("cam_orig");
  for (int32_t n = 0; n < M; ++n) std::printf(" %d", P.cam_orig[n]);
  std::printf("\n");
  for (int32_t l = 0; l < L; ++l) {
    const int32_t nt = P.nt[l];
    const uint8_t* z = P.tile_nz.data() + P.rcs_off[l] / (64 * 64);
    std::printf("block %d %d", l, nt);
    for (int32_t i = 0; i < nt; ++i)
      for (int32_t j = 0; j <= i; ++j) std::printf(" %d", z[i * (i + 1) / 2 + j]);
    std::printf("\n");
  }
  std::vector<int32_t> all(L);
  for (int32_t l = 0; l < L; ++l) all[l] = l;
  std::printf("tasks %zu\n", rpba::dataflow_order(P, all).size());
  return 0;
}
