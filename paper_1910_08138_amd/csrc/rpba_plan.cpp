// Host-side planning of the device data layout.  See rpba_plan.hpp.
#include "rpba_plan.hpp"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <queue>
#include <tuple>

namespace rpba {

namespace {

// Position of every camera inside its sub-block: reverse Cuthill-McKee order
// of the sub-block's co-visibility graph (two cameras are adjacent if they
// observe a common point).  Neighbouring cameras get neighbouring positions,
// so the reduced camera system of the sub-block has its nonzero 6 x 6 blocks
// in a band and its Cholesky factor stays zero outside that band.  Each
// connected part starts at an unvisited camera of least degree; neighbours
// are taken by ascending degree, then by caller order.
std::vector<int32_t> covisibility_rcm(int32_t M, int32_t N, int32_t K, int32_t L, const int32_t* obs_cam,
                                      const int32_t* obs_pt, const int32_t* cam_block, const std::vector<int32_t>& loc,
                                      const std::vector<int32_t>& blk_cam_off) {
  // adjacency bit matrices, one per sub-block, indexed by loc
  std::vector<int64_t> mat_off(L + 1, 0);
  for (int32_t l = 0; l < L; ++l) {
    const int64_t n = blk_cam_off[l + 1] - blk_cam_off[l];
    mat_off[l + 1] = mat_off[l] + n * ((n + 63) / 64);
  }
  std::vector<uint64_t> adj(mat_off[L], 0);
  auto words = [&](int32_t l) { return (int64_t)(blk_cam_off[l + 1] - blk_cam_off[l] + 63) / 64; };
  {
    std::vector<int32_t> off(N + 1, 0), cams(K);
    for (int32_t k = 0; k < K; ++k) off[obs_pt[k] + 1]++;
    for (int32_t j = 0; j < N; ++j) off[j + 1] += off[j];
    std::vector<int32_t> at(off.begin(), off.end() - 1);
    for (int32_t k = 0; k < K; ++k) cams[at[obs_pt[k]]++] = obs_cam[k];
    for (int32_t j = 0; j < N; ++j)
      for (int32_t a = off[j]; a < off[j + 1]; ++a)
        for (int32_t b = off[j]; b < off[j + 1]; ++b) {
          const int32_t ca = cams[a], cb = cams[b];
          if (a == b || cam_block[ca] != cam_block[cb]) continue;
          const int32_t l = cam_block[ca];
          adj[mat_off[l] + loc[ca] * words(l) + loc[cb] / 64] |= 1ull << (loc[cb] % 64);
        }
  }
  std::vector<int32_t> pos(M);
  std::vector<int32_t> blk_cam(M);  // caller index by (sub-block, loc)
  for (int32_t i = 0; i < M; ++i) blk_cam[blk_cam_off[cam_block[i]] + loc[i]] = i;
  for (int32_t l = 0; l < L; ++l) {
    const int32_t n = blk_cam_off[l + 1] - blk_cam_off[l];
    const int64_t W = words(l);
    const uint64_t* A = adj.data() + mat_off[l];
    std::vector<int32_t> deg(n, 0), order, nb;
    for (int32_t u = 0; u < n; ++u)
      for (int64_t w = 0; w < W; ++w) deg[u] += __builtin_popcountll(A[u * W + w]);
    std::vector<char> seen(n, 0);
    order.reserve(n);
    while ((int32_t)order.size() < n) {
      int32_t s0 = -1;
      for (int32_t u = 0; u < n; ++u)
        if (!seen[u] && (s0 < 0 || deg[u] < deg[s0])) s0 = u;
      seen[s0] = 1;
      size_t head = order.size();
      order.push_back(s0);
      while (head < order.size()) {
        const int32_t u = order[head++];
        nb.clear();
        for (int64_t w = 0; w < W; ++w)
          for (uint64_t bits = A[u * W + w]; bits; bits &= bits - 1) {
            const int32_t v = (int32_t)(w * 64 + __builtin_ctzll(bits));
            if (!seen[v]) nb.push_back(v);
          }
        std::sort(nb.begin(), nb.end(), [&](int32_t x, int32_t y) { return deg[x] != deg[y] ? deg[x] < deg[y] : x < y; });
        for (int32_t v : nb) {
          seen[v] = 1;
          order.push_back(v);
        }
      }
    }
    for (int32_t q = 0; q < n; ++q) pos[blk_cam[blk_cam_off[l] + order[n - 1 - q]]] = q;
  }
  return pos;
}

}  // namespace

uint64_t topology_key(int32_t M, int32_t N, int32_t K, int32_t L, const int32_t* obs_cam, const int32_t* obs_pt,
                      const int32_t* cam_block, int32_t tile, int32_t np) {
  // FNV-1a over sizes and the three index arrays
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  mix((uint64_t)M);
  mix((uint64_t)N);
  mix((uint64_t)K);
  mix((uint64_t)L);
  mix((uint64_t)tile);
  mix((uint64_t)np);
  for (int32_t k = 0; k < K; ++k) mix(((uint64_t)(uint32_t)obs_cam[k] << 32) | (uint32_t)obs_pt[k]);
  for (int32_t i = 0; i < M; ++i) mix((uint64_t)(uint32_t)cam_block[i]);
  return h;
}

std::string build_plan(int32_t M, int32_t N, int32_t K, int32_t L, const int32_t* obs_cam, const int32_t* obs_pt,
                       const int32_t* cam_block, int32_t tile, int32_t np, Plan& P) {
  if (np != 6 && np != 8) return "6 or 8 parameters per camera";
  if (M <= 0 || N <= 0 || K <= 0 || L <= 0) return "M, N, K and L must be positive";
  if (M >= (1 << 20)) return "at most 2^20 - 1 cameras";
  if (N >= (1 << 28)) return "at most 2^28 - 1 points";
  if (L >= (1 << 15)) return "at most 2^15 - 1 sub-blocks";
  if (tile != 32 && tile != 64) return "Cholesky tile must be 32 or 64";
  if (!obs_cam || !obs_pt || !cam_block) return "topology arrays must be non-NULL host pointers";
  P = Plan();
  P.np = np;
  P.M = M;
  P.N = N;
  P.K = K;
  P.L = L;
  P.T = tile;
  for (int32_t i = 0; i < M; ++i)
    if (cam_block[i] < 0 || cam_block[i] >= L) return "cam_block out of range at camera " + std::to_string(i);
  std::vector<int32_t> ccount(M, 0), pcount(N, 0);
  for (int32_t k = 0; k < K; ++k) {
    if (obs_cam[k] < 0 || obs_cam[k] >= M) return "obs_cam out of range at observation " + std::to_string(k);
    if (obs_pt[k] < 0 || obs_pt[k] >= N) return "obs_pt out of range at observation " + std::to_string(k);
    ccount[obs_cam[k]]++;
    pcount[obs_pt[k]]++;
  }
  for (int32_t i = 0; i < M; ++i)
    if (ccount[i] < 1) return "camera " + std::to_string(i) + " has no observation";
  for (int32_t j = 0; j < N; ++j)
    if (pcount[j] < 2) return "point " + std::to_string(j) + " has fewer than 2 observations";

  // cameras grouped by sub-block
  P.blk_cam_off.assign(L + 1, 0);
  for (int32_t i = 0; i < M; ++i) P.blk_cam_off[cam_block[i] + 1]++;
  for (int32_t l = 0; l < L; ++l) {
    if (P.blk_cam_off[l + 1] == 0) return "sub-block " + std::to_string(l) + " has no camera";
    P.blk_cam_off[l + 1] += P.blk_cam_off[l];
  }
  P.cam_orig.resize(M);
  P.cam_blk.resize(M);
  std::vector<int32_t> cam_new(M);
  {
    // loc: rank of a camera among the cameras of its sub-block, caller order
    std::vector<int32_t> loc(M), fill(L, 0);
    for (int32_t i = 0; i < M; ++i) loc[i] = fill[cam_block[i]]++;
    const std::vector<int32_t> rcm = covisibility_rcm(M, N, K, L, obs_cam, obs_pt, cam_block, loc, P.blk_cam_off);
    for (int32_t i = 0; i < M; ++i) {
      const int32_t n = P.blk_cam_off[cam_block[i]] + rcm[i];
      P.cam_orig[n] = i;
      cam_new[i] = n;
      P.cam_blk[n] = cam_block[i];
    }
  }
  for (int32_t l = 0; l < L; ++l) P.max_blk_cams = std::max(P.max_blk_cams, P.blk_cam_off[l + 1] - P.blk_cam_off[l]);
  if (np * P.max_blk_cams > 255 * tile) return "sub-block too large for the Cholesky tiling";

  // points ordered by their lowest sub-block and, inside it, by their first
  // camera (cameras of a sub-block are in the caller's order, which for image
  // blocks follows the flight path): neighbouring points then share cameras,
  // so a wave's gathers of camera data and copy records hit the same lines
  std::vector<int32_t> owner(N, L), first(N, M);
  for (int32_t k = 0; k < K; ++k) {
    const int32_t j = obs_pt[k], l = cam_block[obs_cam[k]];
    if (l < owner[j] || (l == owner[j] && cam_new[obs_cam[k]] < first[j])) {
      owner[j] = l;
      first[j] = cam_new[obs_cam[k]];
    }
  }
  P.pt_orig.resize(N);
  std::vector<int32_t>& pt_new = P.pt_new;
  pt_new.assign(N, 0);
  {
    std::vector<int32_t> cnt(M + 1, 0);
    for (int32_t j = 0; j < N; ++j) cnt[first[j] + 1]++;
    for (int32_t i = 0; i < M; ++i) cnt[i + 1] += cnt[i];
    for (int32_t j = 0; j < N; ++j) P.pt_orig[cnt[first[j]]++] = j;
    // inside each intersection workgroup, the points with more observations
    // first: a wave's lanes then walk observation lists of similar length
    for (int32_t b = 0; b < N; b += INT_WG) {
      const int32_t e = std::min(N, b + INT_WG);
      std::stable_sort(P.pt_orig.begin() + b, P.pt_orig.begin() + e,
                       [&](int32_t x, int32_t y) { return pcount[x] > pcount[y]; });
    }
    for (int32_t n = 0; n < N; ++n) pt_new[P.pt_orig[n]] = n;
  }

  // observations in (sub-block, point, camera) order
  std::vector<std::pair<uint64_t, int32_t>> keys(K);
  for (int32_t k = 0; k < K; ++k) {
    uint64_t l = (uint64_t)cam_block[obs_cam[k]];
    keys[k] = {(l << 48) | ((uint64_t)pt_new[obs_pt[k]] << 20) | (uint64_t)cam_new[obs_cam[k]], k};
  }
  std::sort(keys.begin(), keys.end());
  P.obs_orig.resize(K);
  P.obs_cam.resize(K);
  P.obs_copy.resize(K);
  P.copy_off.clear();
  P.copy_pt.clear();
  P.copy_blk.clear();
  P.blk_copy_off.assign(L + 1, 0);
  for (int32_t k = 0; k < K; ++k) {
    uint64_t key = keys[k].first;
    P.obs_orig[k] = keys[k].second;
    P.obs_cam[k] = (int32_t)(key & ((1u << 20) - 1));
    int32_t pt = (int32_t)((key >> 20) & ((1u << 28) - 1));
    int32_t l = (int32_t)(key >> 48);
    if (k > 0 && (keys[k - 1].first >> 20) == (key >> 20)) {
      if (P.obs_cam[k - 1] == P.obs_cam[k])
        return "repeated (camera, point) pair at observation " + std::to_string(keys[k].second);
    } else {
      P.copy_off.push_back(k);
      P.copy_pt.push_back(pt);
      P.copy_blk.push_back(l);
      P.blk_copy_off[l + 1]++;
    }
    P.obs_copy[k] = (int32_t)P.copy_off.size() - 1;
  }
  keys.clear();
  keys.shrink_to_fit();
  P.NC = (int64_t)P.copy_pt.size();
  P.copy_off.push_back(K);
  for (int32_t l = 0; l < L; ++l) P.blk_copy_off[l + 1] += P.blk_copy_off[l];

  // copies of each point (ascending sub-block because copies are (l, pt) sorted)
  P.pt_copy_off.assign(N + 1, 0);
  for (int64_t c = 0; c < P.NC; ++c) P.pt_copy_off[P.copy_pt[c] + 1]++;
  for (int32_t j = 0; j < N; ++j) P.pt_copy_off[j + 1] += P.pt_copy_off[j];
  P.pt_copies.resize(P.NC);
  {
    std::vector<int32_t> fill(P.pt_copy_off.begin(), P.pt_copy_off.end() - 1);
    for (int64_t c = 0; c < P.NC; ++c) P.pt_copies[fill[P.copy_pt[c]]++] = (int32_t)c;
  }

  // point-major observation stream of the intersection and the cameras of
  // each of its workgroups
  P.pm_off.assign(N + 1, 0);
  P.pm_k.resize(K);
  P.pm_pos.resize(K);
  P.pm_cam.resize(K);
  {
    int32_t i = 0;
    for (int32_t j = 0; j < N; ++j) {
      P.pm_off[j] = i;
      for (int32_t cc = P.pt_copy_off[j]; cc < P.pt_copy_off[j + 1]; ++cc) {
        const int32_t c = P.pt_copies[cc];
        for (int32_t k = P.copy_off[c]; k < P.copy_off[c + 1]; ++k) {
          P.pm_k[i] = k;
          P.pm_pos[k] = i;
          P.pm_cam[i] = k + 1 == P.copy_off[c + 1] ? PM_LAST : 0;
          ++i;
        }
      }
    }
    P.pm_off[N] = i;
    const int32_t nwg = (N + INT_WG - 1) / INT_WG;
    P.iwg_cam_off.assign(nwg + 1, 0);
    P.iwg_cams.clear();
    std::vector<int32_t> stamp(M, -1), slot(M, 0);
    for (int32_t w = 0; w < nwg; ++w) {
      const int32_t j0 = w * INT_WG, j1 = std::min(N, j0 + INT_WG);
      int32_t n = 0;
      for (int32_t q = P.pm_off[j0]; q < P.pm_off[j1]; ++q) {
        const int32_t cam = P.obs_cam[P.pm_k[q]];
        if (stamp[cam] != w) {
          stamp[cam] = w;
          if (n < INT_CAM_CAP) {
            slot[cam] = n++;
            P.iwg_cams.push_back(cam);
          } else {
            slot[cam] = PM_GLOBAL | cam;
          }
        }
        P.pm_cam[q] |= slot[cam];
      }
      P.iwg_cam_off[w + 1] = (int32_t)P.iwg_cams.size();
    }
  }

  // observations of each camera (ascending LM index)
  P.cam_obs_off.assign(M + 1, 0);
  for (int32_t k = 0; k < K; ++k) P.cam_obs_off[P.obs_cam[k] + 1]++;
  for (int32_t i = 0; i < M; ++i) {
    P.max_cam_obs = std::max(P.max_cam_obs, P.cam_obs_off[i + 1]);
    P.cam_obs_off[i + 1] += P.cam_obs_off[i];
  }
  P.cam_obs.resize(K);
  {
    std::vector<int32_t> fill(P.cam_obs_off.begin(), P.cam_obs_off.end() - 1);
    for (int32_t k = 0; k < K; ++k) P.cam_obs[fill[P.obs_cam[k]]++] = k;
  }
  P.cam_obs_c.resize(K);
  for (int32_t q = 0; q < K; ++q) P.cam_obs_c[q] = P.obs_copy[P.cam_obs[q]];

  // neighbour lists: cameras of the same sub-block sharing a point copy, local index <= own
  std::vector<std::vector<int32_t>> nb(M);
  for (int32_t i = 0; i < M; ++i) nb[i].push_back(i - P.blk_cam_off[P.cam_blk[i]]);
  for (int64_t c = 0; c < P.NC; ++c) {
    int32_t b = P.copy_off[c], e = P.copy_off[c + 1];
    int32_t base = P.blk_cam_off[P.copy_blk[c]];
    for (int32_t k1 = b; k1 < e; ++k1)
      for (int32_t k2 = b; k2 < k1; ++k2) {
        // obs of a copy are sorted by camera, so obs_cam[k2] < obs_cam[k1]
        nb[P.obs_cam[k1]].push_back(P.obs_cam[k2] - base);
      }
  }
  P.nb_off.assign(M + 1, 0);
  for (int32_t i = 0; i < M; ++i) {
    std::sort(nb[i].begin(), nb[i].end());
    nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
    P.nb_off[i + 1] = P.nb_off[i] + (int32_t)nb[i].size();
    P.max_nb = std::max(P.max_nb, (int32_t)nb[i].size());
  }
  P.nb_cam.resize(P.nb_off[M]);
  for (int32_t i = 0; i < M; ++i) std::copy(nb[i].begin(), nb[i].end(), P.nb_cam.begin() + P.nb_off[i]);

  // block-sparse pattern with both triangles (rows by internal camera)
  {
    std::vector<std::vector<int32_t>> full(M);
    for (int32_t i = 0; i < M; ++i) {
      int32_t base = P.blk_cam_off[P.cam_blk[i]];
      for (int32_t a2 : nb[i]) {
        full[i].push_back(a2);
        int32_t i2 = base + a2;
        if (i2 != i) full[i2].push_back(i - base);
      }
    }
    P.bsr_row_off.assign(M + 1, 0);
    for (int32_t i = 0; i < M; ++i) {
      std::sort(full[i].begin(), full[i].end());
      P.bsr_row_off[i + 1] = P.bsr_row_off[i] + (int32_t)full[i].size();
    }
    P.nbsr = P.bsr_row_off[M];
    P.bsr_col.resize(P.nbsr);
    for (int32_t i = 0; i < M; ++i) std::copy(full[i].begin(), full[i].end(), P.bsr_col.begin() + P.bsr_row_off[i]);
    P.bsr_tr.resize(P.nbsr);
    for (int32_t i = 0; i < M; ++i) {
      int32_t base = P.blk_cam_off[P.cam_blk[i]];
      int32_t ai = i - base;
      for (int32_t q = P.bsr_row_off[i]; q < P.bsr_row_off[i + 1]; ++q) {
        int32_t i2 = base + P.bsr_col[q];
        const int32_t* b = P.bsr_col.data() + P.bsr_row_off[i2];
        const int32_t* e = P.bsr_col.data() + P.bsr_row_off[i2 + 1];
        const int32_t* f = std::lower_bound(b, e, ai);
        P.bsr_tr[q] = (int32_t)(f - P.bsr_col.data());
      }
    }
  }

  // pair blocks and their observation pairs
  {
    const int64_t NPB = (int64_t)P.nb_cam.size();
    P.pb_row.resize(NPB);
    for (int32_t i = 0; i < M; ++i)
      for (int32_t q = P.nb_off[i]; q < P.nb_off[i + 1]; ++q) P.pb_row[q] = i;
    auto pb_of = [&](int32_t i1, int32_t a2) -> int32_t {
      const int32_t* b = P.nb_cam.data() + P.nb_off[i1];
      const int32_t* e = P.nb_cam.data() + P.nb_off[i1 + 1];
      return (int32_t)(std::lower_bound(b, e, a2) - P.nb_cam.data());
    };
    std::vector<int64_t> cnt(NPB + 1, 0);
    for (int64_t c = 0; c < P.NC; ++c) {
      int32_t b = P.copy_off[c], e = P.copy_off[c + 1], base = P.blk_cam_off[P.copy_blk[c]];
      for (int32_t k1 = b; k1 < e; ++k1)
        for (int32_t k2 = b; k2 <= k1; ++k2) cnt[pb_of(P.obs_cam[k1], P.obs_cam[k2] - base) + 1]++;
    }
    for (int64_t q = 0; q < NPB; ++q) cnt[q + 1] += cnt[q];
    P.pb_ent_off = cnt;
    P.pb_ent.resize(3 * (size_t)cnt[NPB]);
    // observations are referred to by their position in their camera's list,
    // where the pair pass reads their weights (in order within a pair block)
    std::vector<int32_t> pos_in_cam(K);
    for (int32_t q = 0; q < K; ++q) pos_in_cam[P.cam_obs[q]] = q;
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t c = 0; c < P.NC; ++c) {
      int32_t b = P.copy_off[c], e = P.copy_off[c + 1], base = P.blk_cam_off[P.copy_blk[c]];
      for (int32_t k1 = b; k1 < e; ++k1)
        for (int32_t k2 = b; k2 <= k1; ++k2) {
          int64_t at = fill[pb_of(P.obs_cam[k1], P.obs_cam[k2] - base)]++;
          P.pb_ent[3 * at] = (int32_t)c;
          P.pb_ent[3 * at + 1] = pos_in_cam[k1];
          P.pb_ent[3 * at + 2] = pos_in_cam[k2];
        }
    }
    P.od_pb.clear();
    for (int64_t q = 0; q < NPB; ++q) {
      int32_t i = P.pb_row[q];
      if (P.nb_cam[q] != i - P.blk_cam_off[P.cam_blk[i]]) P.od_pb.push_back((int32_t)q);
    }
    // by the number of rounds a lane group of the pair pass needs, most
    // first: the pair blocks of a wave take the same number of rounds (a wave
    // lasts as long as its longest) and the long ones start early; inside a
    // class the blocks keep their order (neighbouring cameras, shared copy
    // records)
    auto rounds = [&](int32_t q) { return (P.pb_ent_off[q + 1] - P.pb_ent_off[q] + PB_LANES - 1) / PB_LANES; };
    std::stable_sort(P.od_pb.begin(), P.od_pb.end(), [&](int32_t a, int32_t b) { return rounds(a) > rounds(b); });
    P.pb_bsr.resize(NPB);
    P.pb_bsr_t.resize(NPB);
    for (int64_t q = 0; q < NPB; ++q) {
      int32_t i = P.pb_row[q];
      int32_t base = P.blk_cam_off[P.cam_blk[i]];
      int32_t a2 = P.nb_cam[q];
      const int32_t* rb = P.bsr_col.data() + P.bsr_row_off[i];
      const int32_t* re = P.bsr_col.data() + P.bsr_row_off[i + 1];
      int32_t pos = (int32_t)(std::lower_bound(rb, re, a2) - P.bsr_col.data());
      P.pb_bsr[q] = pos;
      P.pb_bsr_t[q] = P.bsr_tr[pos];
      (void)base;
    }
  }

  // dense tiled reduced camera systems
  const int64_t T2 = (int64_t)tile * tile;
  P.nt.resize(L);
  P.rcs_off.resize(L);
  P.diag_off.resize(L);
  P.vec_off.resize(L);
  P.nt_max = 0;
  for (int32_t l = 0; l < L; ++l) {
    int32_t n6 = np * (P.blk_cam_off[l + 1] - P.blk_cam_off[l]);
    int32_t nt = (n6 + tile - 1) / tile;
    P.nt[l] = nt;
    P.nt_max = std::max(P.nt_max, nt);
    P.rcs_off[l] = P.rcs_total;
    P.rcs_total += ((int64_t)nt * (nt + 1) / 2 + nt) * T2;  // lower triangle + right-hand-side tile row
    P.diag_off[l] = P.diag_total;
    P.diag_total += (int64_t)nt * T2;
    P.vec_off[l] = P.vec_total;
    P.vec_total += (int64_t)nt * tile;
  }
  // tiles of each factor that can be nonzero: the tiles touched by an np x np
  // block of S (a camera's np rows may straddle two tiles), the diagonal
  // tiles, then the fill of a Cholesky factorisation by tiles; the
  // right-hand-side tile row is full
  P.tile_nz.assign(P.rcs_total / T2, 0);
  for (int32_t l = 0; l < L; ++l) {
    const int32_t nt = P.nt[l];
    uint8_t* z = P.tile_nz.data() + P.rcs_off[l] / T2;
    auto at = [&](int32_t i, int32_t j) -> uint8_t& { return i >= j ? z[i * (i + 1) / 2 + j] : z[j * (j + 1) / 2 + i]; };
    for (int32_t i = 0; i < nt; ++i) at(i, i) = 1;
    for (int32_t j = 0; j < nt; ++j) at(nt, j) = 1;
    for (int32_t c = P.blk_cam_off[l]; c < P.blk_cam_off[l + 1]; ++c) {
      const int32_t a = c - P.blk_cam_off[l];
      for (int32_t q = P.nb_off[c]; q < P.nb_off[c + 1]; ++q) {
        const int32_t b = P.nb_cam[q];
        for (int32_t ra : {np * a / tile, (np * a + np - 1) / tile})
          for (int32_t rb : {np * b / tile, (np * b + np - 1) / tile}) at(ra, rb) = 1;
      }
    }
    std::vector<int32_t> rows;
    for (int32_t k = 0; k < nt; ++k) {
      rows.clear();
      for (int32_t i = k + 1; i < nt; ++i)
        if (at(i, k)) rows.push_back(i);
      for (size_t x = 0; x < rows.size(); ++x)
        for (size_t y = 0; y <= x; ++y) at(rows[x], rows[y]) = 1;
    }
  }
  // larger sub-blocks first: their tiles carry the longest dependency chains
  std::vector<int32_t> order(L);
  for (int32_t l = 0; l < L; ++l) order[l] = l;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return P.nt[a] > P.nt[b]; });
  P.pot_off.assign(P.nt_max + 1, 0);
  P.fwd_off.assign(P.nt_max + 1, 0);
  P.upd_off.assign(P.nt_max + 1, 0);
  P.pot_items.clear();
  P.fwd_items.clear();
  P.upd_items.clear();
  for (int32_t k = 0; k < P.nt_max; ++k) {
    for (int32_t l : order)
      if (P.nt[l] > k) P.pot_items.push_back((l << 16) | (k << 8) | k);
    P.pot_off[k + 1] = (int64_t)P.pot_items.size();
    for (int32_t l : order) {
      int32_t nt = P.nt[l];
      if (nt <= k) continue;
      for (int32_t i = k + 1; i <= nt; ++i) P.fwd_items.push_back((l << 16) | (i << 8) | k);
    }
    P.fwd_off[k + 1] = (int64_t)P.fwd_items.size();
    for (int32_t l : order) {
      int32_t nt = P.nt[l];
      for (int32_t j = k + 1; j < nt; ++j)
        for (int32_t i = j; i <= nt; ++i) P.upd_items.push_back((l << 16) | (i << 8) | j);
    }
    P.upd_off[k + 1] = (int64_t)P.upd_items.size();
  }
  // backward launches, step k (descending): items (l, k, j), j <= k
  P.bwd_off.assign(P.nt_max + 1, 0);
  P.bwd_items.clear();
  for (int32_t s = 0; s < P.nt_max; ++s) {
    int32_t k = P.nt_max - 1 - s;
    for (int32_t l = 0; l < L; ++l) {
      if (P.nt[l] <= k) continue;
      for (int32_t j = 0; j <= k; ++j) P.bwd_items.push_back((l << 16) | (k << 8) | j);
    }
    P.bwd_off[s + 1] = (int64_t)P.bwd_items.size();
  }
  P.blk_pcg.assign(L, 0);
  P.key = topology_key(M, N, K, L, obs_cam, obs_pt, cam_block, tile, np);
  return "";
}

// Workgroups take the tasks in list order, and a task holds its workgroup
// from the moment it is taken: it sums its tile products (k < j with both
// tiles nonzero) as their inputs appear, then factors the diagonal tile or,
// below the diagonal, waits for the diagonal tile and solves.  The tiles on
// the chain diagonal (j) -> panel (j + 1, j) -> diagonal (j + 1) set the
// length of the launch, and each of them sums its products before its last
// input arrives, so a good order
// takes every task at about the latest time that still lets it finish when
// the chain needs it: finish time = depth on the chain (diagonal (j) at 2j,
// tiles below it at 2j + 1, the chains of all sub-blocks ending together)
// times the half-column time, start = finish - own work.  Tasks are released
// in that order, each only after its dependencies (Kahn's algorithm), so a
// task never waits for a task further down the list and the launch cannot
// deadlock.  The costs are measured per-task times of the 64-wide tiles, in
// microseconds; only their ratios matter.
std::vector<int32_t> dataflow_order(const Plan& P, const std::vector<int32_t>& blocks) {
  constexpr double kHalfColumn = 14.0, kProduct = 3.0, kFactor = 17.0, kSolve = 5.0;
  const int64_t T2 = (int64_t)P.T * P.T;
  struct Task {
    int32_t l, i, j;
  };
  // task ids: the tiles of the listed sub-blocks in storage order
  std::vector<int64_t> base(blocks.size() + 1, 0);
  for (size_t b = 0; b < blocks.size(); ++b) {
    const int64_t n = P.nt[blocks[b]];
    base[b + 1] = base[b] + n * (n + 1) / 2 + n;
  }
  auto id = [&](size_t b, int32_t i, int32_t j) { return base[b] + (int64_t)i * (i + 1) / 2 + j; };
  const int64_t ntile = base.back();
  std::vector<Task> tasks(ntile);
  std::vector<char> live(ntile, 0);
  std::vector<double> prio(ntile);
  std::vector<int32_t> indeg(ntile, 0);
  std::vector<std::vector<int64_t>> users(ntile);
  for (size_t b = 0; b < blocks.size(); ++b) {
    const int32_t l = blocks[b], n = P.nt[l];
    const uint8_t* z = P.tile_nz.data() + P.rcs_off[l] / T2;
    auto nz = [&](int32_t i, int32_t j) { return z[i * (i + 1) / 2 + j] != 0; };
    // a nonzero sub-diagonal tile (j, j - 1) of the factor is solved by the
    // task of diagonal tile j (fused): its own task only sums its products
    // (partial), and tile (j, j - 1) is ready when the diagonal task has
    // solved it
    auto fused = [&](int32_t j) { return j >= 1 && j < n && nz(j, j - 1); };
    auto producer = [&](int32_t r, int32_t c) { return r == c + 1 && fused(r) ? id(b, r, r) : id(b, r, c); };
    for (int32_t j = 0; j < n; ++j)
      for (int32_t i = j; i <= n; ++i) {
        if (!nz(i, j)) continue;
        const int64_t t = id(b, i, j);
        tasks[t] = {l, i, j};
        live[t] = 1;
        const bool partial = i == j + 1 && fused(i);
        const bool fd = i == j && fused(j);
        int32_t nprod = 0, ndep = 0;
        for (int32_t k = 0; k < (fd ? j - 1 : j); ++k) {
          if (!nz(i, k) || !nz(j, k)) continue;
          ++nprod;
          users[producer(i, k)].push_back(t);
          ++ndep;
          if (i != j) {
            users[producer(j, k)].push_back(t);
            ++ndep;
          }
        }
        if (fd) {
          // the partial sums of tile (j, j - 1) and the inverse of diagonal
          // tile j - 1; then one more product, with the solved tile
          users[id(b, j, j - 1)].push_back(t);
          users[id(b, j - 1, j - 1)].push_back(t);
          ndep += 2;
          ++nprod;
        } else if (i != j && !partial) {
          users[id(b, j, j)].push_back(t);
          ++ndep;
        }
        indeg[t] = ndep;
        // (the partial sums of tile (j + 1, j) are needed when diagonal tile
        // j is done, like the inverse it publishes)
        const int depth = i == j || partial ? 2 * j : 2 * j + 1;
        const double own = i == j ? kFactor + (fd ? kSolve : 0.0) : partial ? 0.0 : kSolve;
        prio[t] = (depth - (2 * n - 1)) * kHalfColumn - (nprod * kProduct + own);
      }
  }
  using Key = std::tuple<double, int32_t, int32_t, int32_t, int64_t>;
  std::priority_queue<Key, std::vector<Key>, std::greater<Key>> ready;
  int64_t nlive = 0;
  for (int64_t t = 0; t < ntile; ++t)
    if (live[t]) {
      ++nlive;
      if (indeg[t] == 0) ready.push({prio[t], tasks[t].l, tasks[t].j, tasks[t].i, t});
    }
  std::vector<int32_t> out;
  out.reserve(nlive);
  std::vector<int64_t> pos(ntile, -1);
  while (!ready.empty()) {
    const int64_t t = std::get<4>(ready.top());
    ready.pop();
    pos[t] = (int64_t)out.size();
    out.push_back((tasks[t].l << 16) | (tasks[t].i << 8) | tasks[t].j);
    for (int64_t u : users[t])
      if (--indeg[u] == 0) ready.push({prio[u], tasks[u].l, tasks[u].j, tasks[u].i, u});
  }
  // every dependency strictly earlier
  bool ok = (int64_t)out.size() == nlive;
  for (int64_t t = 0; ok && t < ntile; ++t)
    for (int64_t u : users[t])
      if (!live[t] || pos[t] < 0 || pos[t] >= pos[u]) ok = false;
  if (!ok) out.clear();
  return out;
}

}  // namespace rpba
