// Sub-block construction by partitioning the visibility graph (paper Sec.
// 5.2).  Host code: the partition is computed once per block, before
// rpba_create, from the observation lists alone.
//
// Graph: one node per camera; two cameras are joined by an edge whose weight
// is the number of points both observe.  Node weight of camera i: the cube
// root of the summed observation counts of the points camera i sees (the
// weighting the paper found to track the adjustment cost best).
//
// Multilevel recursive bisection, written for this library:
//   * coarsening by heavy-edge matching (random visiting order, a matched
//     pair may not outweigh 1.5 / 40 of the graph) until about 40 nodes
//     remain or a level shrinks the graph by less than a tenth;
//   * initial bisection of the coarsest graph by greedy graph growing from
//     several seeds (one of them a peripheral node), each refined, the best
//     kept;
//   * projection back level by level, each followed by Fiduccia-Mattheyses
//     boundary refinement (moves by largest cut gain under the balance
//     bound, hill climbing with roll-back to the best prefix);
//   * the two halves are partitioned recursively into floor(L/2) and
//     ceil(L/2) parts with node-weight targets in that ratio.
// An optional pass then balances a cost model per part, c3 n_l^3 + c1 K_l
// (n_l cameras, K_l observations), by moving boundary cameras out of the
// most expensive part while that lowers the largest cost.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <queue>
#include <random>
#include <vector>

#include "rpba.h"

namespace rpba {

// sets the message rpba_last_error returns (defined with the C-ABI layer)
rpba_status report_error(rpba_status s, const char* msg);

namespace {

struct Graph {
  int32_t n = 0;
  std::vector<int64_t> xadj;  // [n + 1]
  std::vector<int32_t> adj;   // neighbours
  std::vector<int64_t> ew;    // edge weights
  std::vector<double> vw;     // node weights
  double total() const { return std::accumulate(vw.begin(), vw.end(), 0.0); }
};

// CSR lists of the observations by point and by camera
struct Incidence {
  std::vector<int32_t> pt_off, pt_cam, cam_off, cam_pt;
};

Incidence incidence(int32_t M, int32_t N, int32_t K, const int32_t* obs_cam, const int32_t* obs_pt) {
  Incidence I;
  I.pt_off.assign(N + 1, 0);
  I.cam_off.assign(M + 1, 0);
  for (int32_t k = 0; k < K; ++k) {
    I.pt_off[obs_pt[k] + 1]++;
    I.cam_off[obs_cam[k] + 1]++;
  }
  for (int32_t j = 0; j < N; ++j) I.pt_off[j + 1] += I.pt_off[j];
  for (int32_t i = 0; i < M; ++i) I.cam_off[i + 1] += I.cam_off[i];
  I.pt_cam.resize(K);
  I.cam_pt.resize(K);
  std::vector<int32_t> a(I.pt_off.begin(), I.pt_off.end() - 1), b(I.cam_off.begin(), I.cam_off.end() - 1);
  for (int32_t k = 0; k < K; ++k) {
    I.pt_cam[a[obs_pt[k]]++] = obs_cam[k];
    I.cam_pt[b[obs_cam[k]]++] = obs_pt[k];
  }
  return I;
}

Graph visibility_graph(int32_t M, const Incidence& I) {
  Graph g;
  g.n = M;
  g.xadj.assign(M + 1, 0);
  g.vw.assign(M, 0.0);
  std::vector<int64_t> acc(M, 0);
  std::vector<int32_t> touched;
  for (int32_t i = 0; i < M; ++i) {
    double s = 0.0;
    touched.clear();
    for (int32_t q = I.cam_off[i]; q < I.cam_off[i + 1]; ++q) {
      const int32_t j = I.cam_pt[q];
      s += (double)(I.pt_off[j + 1] - I.pt_off[j]);
      for (int32_t r = I.pt_off[j]; r < I.pt_off[j + 1]; ++r) {
        const int32_t c = I.pt_cam[r];
        if (c == i) continue;
        if (acc[c] == 0) touched.push_back(c);
        acc[c] += 1;
      }
    }
    g.vw[i] = std::cbrt(s);
    std::sort(touched.begin(), touched.end());
    for (int32_t c : touched) {
      g.adj.push_back(c);
      g.ew.push_back(acc[c]);
      acc[c] = 0;
    }
    g.xadj[i + 1] = (int64_t)g.adj.size();
  }
  return g;
}

// subgraph induced by the nodes with sel[u] == s, local numbering in `ids`
Graph induced(const Graph& g, const std::vector<uint8_t>& sel, uint8_t s, std::vector<int32_t>& ids) {
  std::vector<int32_t> loc(g.n, -1);
  ids.clear();
  for (int32_t u = 0; u < g.n; ++u)
    if (sel[u] == s) {
      loc[u] = (int32_t)ids.size();
      ids.push_back(u);
    }
  Graph h;
  h.n = (int32_t)ids.size();
  h.xadj.assign(h.n + 1, 0);
  h.vw.resize(h.n);
  for (int32_t a = 0; a < h.n; ++a) {
    const int32_t u = ids[a];
    h.vw[a] = g.vw[u];
    for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e)
      if (loc[g.adj[e]] >= 0) {
        h.adj.push_back(loc[g.adj[e]]);
        h.ew.push_back(g.ew[e]);
      }
    h.xadj[a + 1] = (int64_t)h.adj.size();
  }
  return h;
}

// heavy-edge matching; cmap[u] = coarse node of u
Graph coarsen(const Graph& g, std::vector<int32_t>& cmap, std::mt19937_64& rng, double max_vw) {
  std::vector<int32_t> perm(g.n);
  std::iota(perm.begin(), perm.end(), 0);
  std::shuffle(perm.begin(), perm.end(), rng);
  std::vector<int32_t> match(g.n, -1);
  for (int32_t u : perm) {
    if (match[u] >= 0) continue;
    int32_t best = -1;
    int64_t bw = -1;
    for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
      const int32_t v = g.adj[e];
      if (match[v] >= 0 || v == u || g.vw[u] + g.vw[v] > max_vw) continue;
      if (g.ew[e] > bw) {
        bw = g.ew[e];
        best = v;
      }
    }
    if (best >= 0) {
      match[u] = best;
      match[best] = u;
    } else {
      match[u] = u;
    }
  }
  cmap.assign(g.n, -1);
  int32_t nc = 0;
  for (int32_t u : perm)
    if (cmap[u] < 0) {
      cmap[u] = nc;
      cmap[match[u]] = nc;
      ++nc;
    }
  Graph c;
  c.n = nc;
  c.xadj.assign(nc + 1, 0);
  c.vw.assign(nc, 0.0);
  std::vector<std::vector<int32_t>> members(nc);
  for (int32_t u = 0; u < g.n; ++u) {
    c.vw[cmap[u]] += g.vw[u];
    members[cmap[u]].push_back(u);
  }
  std::vector<int64_t> acc(nc, 0);
  std::vector<int32_t> touched;
  for (int32_t a = 0; a < nc; ++a) {
    touched.clear();
    for (int32_t u : members[a])
      for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
        const int32_t b = cmap[g.adj[e]];
        if (b == a) continue;
        if (acc[b] == 0) touched.push_back(b);
        acc[b] += g.ew[e];
      }
    std::sort(touched.begin(), touched.end());
    for (int32_t b : touched) {
      c.adj.push_back(b);
      c.ew.push_back(acc[b]);
      acc[b] = 0;
    }
    c.xadj[a + 1] = (int64_t)c.adj.size();
  }
  return c;
}

int64_t cut_of(const Graph& g, const std::vector<uint8_t>& side) {
  int64_t c = 0;
  for (int32_t u = 0; u < g.n; ++u)
    for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e)
      if (side[g.adj[e]] != side[u]) c += g.ew[e];
  return c / 2;
}

struct Bounds {
  double cap[2];  // largest allowed weight of each side
};

double violation(const double pw[2], const Bounds& b) { return std::max(pw[0] / b.cap[0], pw[1] / b.cap[1]); }

// Fiduccia-Mattheyses refinement of a bisection, `passes` passes at most
void fm_refine(const Graph& g, std::vector<uint8_t>& side, const Bounds& b, int passes) {
  const int32_t n = g.n;
  std::vector<int64_t> ext(n, 0), in(n, 0);
  double pw[2] = {0.0, 0.0};
  for (int32_t u = 0; u < n; ++u) {
    pw[side[u]] += g.vw[u];
    for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) (side[g.adj[e]] != side[u] ? ext[u] : in[u]) += g.ew[e];
  }
  int64_t cut = 0;
  for (int32_t u = 0; u < n; ++u) cut += ext[u];
  cut /= 2;
  auto move = [&](int32_t v) {
    const uint8_t from = side[v], to = 1 - from;
    side[v] = to;
    pw[from] -= g.vw[v];
    pw[to] += g.vw[v];
    cut -= ext[v] - in[v];
    std::swap(ext[v], in[v]);
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
      const int32_t u = g.adj[e];
      if (side[u] == to) {
        ext[u] -= g.ew[e];
        in[u] += g.ew[e];
      } else {
        ext[u] += g.ew[e];
        in[u] -= g.ew[e];
      }
    }
  };
  std::vector<uint8_t> locked(n, 0);
  std::vector<int32_t> moved;
  for (int pass = 0; pass < passes; ++pass) {
    using Item = std::pair<int64_t, int32_t>;  // (gain, -node): largest gain, then lowest index
    std::priority_queue<Item> heap;
    std::fill(locked.begin(), locked.end(), 0);
    for (int32_t u = 0; u < n; ++u)
      if (ext[u] > 0) heap.push(Item(ext[u] - in[u], -u));
    moved.clear();
    double best_v = std::max(violation(pw, b), 1.0);
    int64_t best_cut = cut;
    size_t best_len = 0;
    int since_best = 0;
    while (!heap.empty() && since_best < 64) {
      const Item it = heap.top();
      heap.pop();
      const int32_t v = -it.second;
      if (locked[v] || it.first != ext[v] - in[v]) continue;
      const uint8_t to = 1 - side[v];
      const double v_now = violation(pw, b);
      double npw[2] = {pw[0], pw[1]};
      npw[side[v]] -= g.vw[v];
      npw[to] += g.vw[v];
      const double v_new = violation(npw, b);
      locked[v] = 1;
      if (v_new > 1.0 && v_new >= v_now) continue;  // would break (or worsen) the balance
      move(v);
      moved.push_back(v);
      for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
        const int32_t u = g.adj[e];
        if (!locked[u] && ext[u] > 0) heap.push(Item(ext[u] - in[u], -u));
      }
      const double vv = std::max(violation(pw, b), 1.0);
      if (vv < best_v || (vv == best_v && cut < best_cut)) {
        best_v = vv;
        best_cut = cut;
        best_len = moved.size();
        since_best = 0;
      } else {
        ++since_best;
      }
    }
    for (size_t q = moved.size(); q > best_len; --q) move(moved[q - 1]);
    if (best_len == 0) break;
  }
}

// greedy graph growing from `seed` until side 0 holds about `target` weight
void grow(const Graph& g, int32_t seed, double target, std::vector<uint8_t>& side) {
  const int32_t n = g.n;
  side.assign(n, 1);
  std::vector<int64_t> conn(n, 0), deg(n, 0);
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) deg[u] += g.ew[e];
  using Item = std::pair<int64_t, int32_t>;
  std::priority_queue<Item> heap;
  double w0 = 0.0;
  int32_t next_free = 0;
  int32_t v = seed;
  while (true) {
    if (v < 0) {  // the region's component is used up: continue at another node
      while (next_free < n && side[next_free] == 0) ++next_free;
      if (next_free >= n) break;
      v = next_free;
    }
    if (w0 > 0.0 && std::fabs(w0 + g.vw[v] - target) >= std::fabs(w0 - target)) break;
    side[v] = 0;
    w0 += g.vw[v];
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
      const int32_t u = g.adj[e];
      if (side[u] == 0) continue;
      conn[u] += g.ew[e];
      heap.push(Item(2 * conn[u] - deg[u], -u));
    }
    v = -1;
    while (!heap.empty()) {
      const Item it = heap.top();
      heap.pop();
      const int32_t u = -it.second;
      if (side[u] == 0 || it.first != 2 * conn[u] - deg[u]) continue;
      v = u;
      break;
    }
  }
}

// a node far from `start` (two breadth-first sweeps)
int32_t peripheral(const Graph& g, int32_t start) {
  int32_t last = start;
  for (int sweep = 0; sweep < 2; ++sweep) {
    std::vector<int32_t> dist(g.n, -1);
    std::queue<int32_t> q;
    q.push(last);
    dist[last] = 0;
    while (!q.empty()) {
      const int32_t u = q.front();
      q.pop();
      last = u;
      for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e)
        if (dist[g.adj[e]] < 0) {
          dist[g.adj[e]] = dist[u] + 1;
          q.push(g.adj[e]);
        }
    }
  }
  return last;
}

// balance bound of a level: the share plus eps, plus the weight of the
// heaviest node of that level at the coarse levels (where a single move
// would otherwise break the bound and freeze the refinement)
Bounds level_bounds(const Graph& g, double W, double f, double eps, bool finest) {
  const double slack = finest ? 0.0 : *std::max_element(g.vw.begin(), g.vw.end());
  Bounds b;
  b.cap[0] = (1.0 + eps) * f * W + slack;
  b.cap[1] = (1.0 + eps) * (1.0 - f) * W + slack;
  return b;
}

// multilevel bisection: side[u] = 0 for a share f of the weight
std::vector<uint8_t> bisect(const Graph& g0, double f, double eps, int passes, std::mt19937_64& rng) {
  const double W = g0.total();
  std::vector<Graph> levels;
  std::vector<std::vector<int32_t>> maps;
  levels.push_back(g0);
  const double max_vw = 1.5 * W / 40.0;
  while (levels.back().n > 40) {
    std::vector<int32_t> cmap;
    Graph c = coarsen(levels.back(), cmap, rng, max_vw);
    if (c.n > 0.9 * levels.back().n) break;
    maps.push_back(std::move(cmap));
    levels.push_back(std::move(c));
  }
  const Graph& gc = levels.back();
  const Bounds b = level_bounds(gc, W, f, eps, levels.size() == 1);
  std::vector<uint8_t> best, side;
  int64_t best_cut = INT64_MAX;
  double best_v = 1e300;
  const int trials = std::min<int32_t>(gc.n, 8);
  for (int t = 0; t < trials; ++t) {
    const int32_t seed = t == 0 ? peripheral(gc, 0) : (int32_t)(rng() % (uint64_t)gc.n);
    grow(gc, seed, f * W, side);
    fm_refine(gc, side, b, passes);
    double pw[2] = {0.0, 0.0};
    for (int32_t u = 0; u < gc.n; ++u) pw[side[u]] += gc.vw[u];
    const double v = std::max(violation(pw, b), 1.0);
    const int64_t c = cut_of(gc, side);
    if (v < best_v || (v == best_v && c < best_cut)) {
      best_v = v;
      best_cut = c;
      best = side;
    }
  }
  for (size_t lv = levels.size() - 1; lv > 0; --lv) {
    const Graph& fine = levels[lv - 1];
    const std::vector<int32_t>& cmap = maps[lv - 1];
    std::vector<uint8_t> fs(fine.n);
    for (int32_t u = 0; u < fine.n; ++u) fs[u] = best[cmap[u]];
    fm_refine(fine, fs, level_bounds(fine, W, f, eps, lv == 1), passes);
    best.swap(fs);
  }
  return best;
}

// every side must hold at least `need` nodes: move the nodes best connected
// to the short side over
void ensure_count(const Graph& g, std::vector<uint8_t>& side, int need0, int need1) {
  for (int s = 0; s < 2; ++s) {
    const int need = s == 0 ? need0 : need1;
    int cnt = 0;
    for (int32_t u = 0; u < g.n; ++u) cnt += side[u] == s;
    while (cnt < need) {
      int32_t best = -1;
      int64_t bc = -1;
      for (int32_t u = 0; u < g.n; ++u) {
        if (side[u] == s) continue;
        int64_t c = 0;
        for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e)
          if (side[g.adj[e]] == s) c += g.ew[e];
        if (c > bc) {
          bc = c;
          best = u;
        }
      }
      side[best] = (uint8_t)s;
      ++cnt;
    }
  }
}

void recurse(const Graph& g, const std::vector<int32_t>& gid, int parts, int first, double eps, int passes,
             std::mt19937_64& rng, int32_t* out) {
  if (parts == 1) {
    for (int32_t u = 0; u < g.n; ++u) out[gid[u]] = first;
    return;
  }
  const int p0 = parts / 2, p1 = parts - p0;
  std::vector<uint8_t> side = bisect(g, (double)p0 / parts, eps, passes, rng);
  ensure_count(g, side, p0, p1);
  for (int s = 0; s < 2; ++s) {
    std::vector<int32_t> ids;
    Graph h = induced(g, side, (uint8_t)s, ids);
    std::vector<int32_t> hg(ids.size());
    for (size_t a = 0; a < ids.size(); ++a) hg[a] = gid[ids[a]];
    recurse(h, hg, s == 0 ? p0 : p1, s == 0 ? first : first + p0, eps, passes, rng, out);
  }
}

// cost-model balancing: boundary cameras leave the most expensive part while
// that lowers the largest cost; among such moves the one adding least cut
void cost_balance(const Graph& g, const std::vector<int64_t>& cam_obs, int parts, double c3, double c1, int32_t* part) {
  std::vector<int64_t> n(parts, 0), k(parts, 0);
  for (int32_t u = 0; u < g.n; ++u) {
    n[part[u]]++;
    k[part[u]] += cam_obs[u];
  }
  auto cost = [&](int64_t nn, int64_t kk) { return c3 * (double)nn * nn * nn + c1 * (double)kk; };
  std::vector<int64_t> to_part(parts, 0);
  std::vector<int32_t> touched;
  for (int32_t iter = 0; iter < 4 * g.n; ++iter) {
    int lmax = 0;
    for (int l = 1; l < parts; ++l)
      if (cost(n[l], k[l]) > cost(n[lmax], k[lmax])) lmax = l;
    const double cmax = cost(n[lmax], k[lmax]);
    if (n[lmax] <= 1) break;
    int32_t bu = -1, bl = -1;
    double bnew = cmax;
    int64_t bdc = INT64_MAX;
    for (int32_t u = 0; u < g.n; ++u) {
      if (part[u] != lmax) continue;
      touched.clear();
      int64_t own = 0;
      for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
        const int l = part[g.adj[e]];
        if (l == lmax) {
          own += g.ew[e];
          continue;
        }
        if (to_part[l] == 0) touched.push_back(l);
        to_part[l] += g.ew[e];
      }
      for (int l : touched) {
        const double a = cost(n[lmax] - 1, k[lmax] - cam_obs[u]);
        const double c = cost(n[l] + 1, k[l] + cam_obs[u]);
        const double nm = std::max(a, c);
        const int64_t dc = own - to_part[l];  // cut change of the move
        if (nm < cmax && (nm < bnew - 1e-12 * cmax || (nm <= bnew + 1e-12 * cmax && dc < bdc))) {
          bnew = nm;
          bdc = dc;
          bu = u;
          bl = l;
        }
      }
      for (int l : touched) to_part[l] = 0;
    }
    if (bu < 0) break;
    n[lmax]--;
    k[lmax] -= cam_obs[bu];
    n[bl]++;
    k[bl] += cam_obs[bu];
    part[bu] = bl;
  }
}

}  // namespace
}  // namespace rpba

extern "C" {

rpba_status rpba_partition_default_options(rpba_partition_options* opt) {
  if (!opt) return rpba::report_error(RPBA_ERR_ARG, "rpba_partition_default_options: NULL options");
  opt->parts = 1;
  opt->imbalance = 0.05;
  opt->min_cams = 0;
  opt->refine_passes = 4;
  opt->cost_cams3 = 0.0;
  opt->cost_obs = 0.0;
  opt->seed = 0;
  return RPBA_OK;
}

rpba_status rpba_partition(int32_t M, int32_t N, int32_t K, const int32_t* obs_cam, const int32_t* obs_pt,
                           const rpba_partition_options* opt, int32_t* cam_block, double* node_weight,
                           double* stats) {
  using namespace rpba;
  if (M < 1 || N < 1 || K < 1) return report_error(RPBA_ERR_ARG, "rpba_partition: M, N and K must be >= 1");
  if (!obs_cam || !obs_pt || !opt || !cam_block)
    return report_error(RPBA_ERR_ARG, "rpba_partition: obs_cam, obs_pt, opt and cam_block must be non-NULL");
  if (opt->parts < 1 || opt->parts > M) return report_error(RPBA_ERR_ARG, "rpba_partition: parts must be in [1, M]");
  if (!(opt->imbalance >= 0.0) || opt->min_cams < 0 || opt->refine_passes < 0 || !(opt->cost_cams3 >= 0.0) ||
      !(opt->cost_obs >= 0.0))
    return report_error(RPBA_ERR_ARG, "rpba_partition: negative imbalance, min_cams, refine_passes or cost coefficient");
  for (int32_t k = 0; k < K; ++k)
    if (obs_cam[k] < 0 || obs_cam[k] >= M || obs_pt[k] < 0 || obs_pt[k] >= N)
      return report_error(RPBA_ERR_ARG, "rpba_partition: observation index out of range");
  int parts = opt->parts;
  if (opt->min_cams > 0) parts = std::max(1, std::min(parts, M / opt->min_cams));
  const Incidence I = incidence(M, N, K, obs_cam, obs_pt);
  const Graph g = visibility_graph(M, I);
  if (node_weight)
    for (int32_t i = 0; i < M; ++i) node_weight[i] = g.vw[i];
  // balance bound per bisection level, so that the bound compounds to
  // about 1 + imbalance over the ceil(log2 parts) levels
  int levels = 0;
  while ((1 << levels) < parts) ++levels;
  const double eps = levels > 0 ? std::pow(1.0 + opt->imbalance, 1.0 / levels) - 1.0 : 0.0;
  std::mt19937_64 rng(opt->seed);
  std::vector<int32_t> gid(M);
  std::iota(gid.begin(), gid.end(), 0);
  recurse(g, gid, parts, 0, eps, opt->refine_passes, rng, cam_block);
  std::vector<int64_t> cam_obs(M);
  for (int32_t i = 0; i < M; ++i) cam_obs[i] = I.cam_off[i + 1] - I.cam_off[i];
  const bool model = opt->cost_cams3 > 0.0 || opt->cost_obs > 0.0;
  if (model && parts > 1) cost_balance(g, cam_obs, parts, opt->cost_cams3, opt->cost_obs, cam_block);
  if (stats) {
    int64_t cut = 0;
    for (int32_t u = 0; u < M; ++u)
      for (int64_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e)
        if (cam_block[g.adj[e]] != cam_block[u]) cut += g.ew[e];
    cut /= 2;
    int64_t tps = 0, copies = 0;
    std::vector<int32_t> seen(parts, -1);
    for (int32_t j = 0; j < N; ++j) {
      int np = 0;
      for (int32_t r = I.pt_off[j]; r < I.pt_off[j + 1]; ++r) {
        const int l = cam_block[I.pt_cam[r]];
        if (seen[l] != j) {
          seen[l] = j;
          ++np;
        }
      }
      copies += np;
      tps += np >= 2;
    }
    std::vector<double> pw(parts, 0.0), pc(parts, 0.0);
    std::vector<int64_t> pn(parts, 0), pk(parts, 0);
    for (int32_t i = 0; i < M; ++i) {
      pw[cam_block[i]] += g.vw[i];
      pn[cam_block[i]]++;
      pk[cam_block[i]] += cam_obs[i];
    }
    for (int l = 0; l < parts; ++l)
      pc[l] = opt->cost_cams3 * (double)pn[l] * pn[l] * pn[l] + opt->cost_obs * (double)pk[l];
    const double wmean = std::accumulate(pw.begin(), pw.end(), 0.0) / parts;
    const double cmean = std::accumulate(pc.begin(), pc.end(), 0.0) / parts;
    stats[0] = parts;
    stats[1] = (double)cut;
    stats[2] = (double)tps;
    stats[3] = (double)copies;
    stats[4] = *std::max_element(pw.begin(), pw.end()) / wmean;
    stats[5] = cmean > 0.0 ? *std::max_element(pc.begin(), pc.end()) / cmean : 0.0;
    stats[6] = (double)*std::min_element(pn.begin(), pn.end());
    stats[7] = (double)*std::max_element(pn.begin(), pn.end());
  }
  return RPBA_OK;
}

}  // extern "C"
