// Host-side tree and per-level plans of HIF-DE; see planner.hpp.
#include "planner.hpp"

#include <algorithm>
#include <stdexcept>

namespace hifde {

std::string check_geom(int dim, int64_t n, int64_t leaf, int skip, Geom* out) {
  if (dim != 2 && dim != 3) return "dim must be 2 or 3";
  if (leaf < 2) return "leaf must be at least 2";
  if (n < 4 || n % leaf != 0) return "leaf must divide n";
  int64_t B = n / leaf;
  if (B < 2 || (B & (B - 1)) != 0) return "n/leaf must be a power of two >= 2";
  if (skip < 0) return "skip_levels must be >= 0";
  int64_t N = 1;
  for (int k = 0; k < dim; ++k) N *= n;
  if (N >= (int64_t(1) << 31)) return "N must be below 2^31";
  Geom g;
  g.dim = dim;
  g.n = n;
  g.m = leaf;
  g.N = N;
  g.skip = skip;
  int L = 0;
  while ((int64_t(1) << L) < B) ++L;
  g.L = L;
  g.stride[0] = 1;
  g.stride[1] = n;
  g.stride[2] = n * n;
  *out = g;
  return "";
}

Planner::Planner(const Geom& g) : g_(g) {
  active_.assign(g_.N, 1);
  grouped_.assign(g_.N, 0);
  loc_.assign(g_.N, -1);
  lv_.resize(g_.L + 1);
}

int64_t Planner::active_count() const {
  int64_t c = 0;
  for (auto a : active_) c += a;
  return c;
}

void Planner::coords(int64_t d, int64_t* x) const {
  for (int k = 0; k < g_.dim; ++k) x[k] = (d / g_.stride[k]) % g_.n;
}

int Planner::sigma(int64_t d, int64_t M) const {
  int64_t x[3];
  coords(d, x);
  int s = 0;
  for (int k = 0; k < g_.dim; ++k) s += is_sep(x[k], M) ? 1 : 0;
  return s;
}

int64_t Planner::box_of(int64_t d, int64_t M) const {
  int64_t x[3];
  coords(d, x);
  int64_t B = g_.n / M, id = 0, mul = 1;
  for (int k = 0; k < g_.dim; ++k) {
    id += (x[k] / M) * mul;
    mul *= B;
  }
  return id;
}

// k * B^dim + lexicographic(box indices), with the separator axis k.
int64_t Planner::group_key(int64_t d, int64_t M) const {
  int64_t x[3];
  coords(d, x);
  int64_t B = g_.n / M, id = 0, mul = 1;
  int axis = 0;
  for (int k = 0; k < g_.dim; ++k) {
    if (is_sep(x[k], M)) axis = k;
    id += (x[k] / M) * mul;
    mul *= B;
  }
  return int64_t(axis) * mul + id;
}

template <class F>
void Planner::for_neighbors(int64_t d, F&& f) const {
  int64_t x[3];
  coords(d, x);
  for (int k = 0; k < g_.dim; ++k) {
    if (x[k] > 0) f(d - g_.stride[k], k, /*up=*/false);
    if (x[k] < g_.n - 1) f(d + g_.stride[k], k, /*up=*/true);
  }
}

static inline int64_t link_ref(int64_t N, int64_t lo, int k) { return N * (1 + k) + lo; }

// ---------------------------------------------------------------------------
// Cells of level l
// ---------------------------------------------------------------------------
void Planner::plan_cells(int l) {
  Level& lev = lv_[l];
  lev.cells.clear();
  lev.maps.clear();
  const bool top = (l == g_.L);
  const int64_t M = top ? g_.n * 2 : (g_.m << l);  // top: no separators
  const int64_t B = top ? 1 : g_.n / M;
  int64_t nbox = 1;
  for (int k = 0; k < g_.dim; ++k) nbox *= B;

  // Interiors: active unknowns with sigma_l == 0, bucketed by box; the
  // ascending scan keeps each bucket sorted.
  std::vector<int32_t> cell_of_box(nbox, -1);
  std::vector<std::vector<int32_t>> bucket(nbox);
  for (int64_t d = 0; d < g_.N; ++d) {
    if (!active_[d]) continue;
    if (!top && sigma(d, M) != 0) continue;
    bucket[top ? 0 : box_of(d, M)].push_back(int32_t(d));
  }
  for (int64_t b = 0; b < nbox; ++b) {
    if (bucket[b].empty()) continue;
    cell_of_box[b] = int32_t(lev.cells.size());
    Cell c;
    c.cid = top ? -1 : b;
    int64_t bb = b, par = 0;
    for (int k = 0; k < g_.dim; ++k) {
      par += bb % B;
      bb /= B;
    }
    c.color = int32_t(par & 1);
    c.p.swap(bucket[b]);
    lev.cells.push_back(std::move(c));
  }

  // Children of each cell (level l-1 cells inside its box).
  std::vector<std::vector<int32_t>> kids(lev.cells.size());
  if (l > 0) {
    Level& prev = lv_[l - 1];
    const int64_t Mp = g_.m << (l - 1);
    const int64_t Bp = g_.n / Mp;
    for (size_t ci = 0; ci < prev.cells.size(); ++ci) {
      int64_t pb = prev.cells[ci].cid, parent_box = 0, mul = 1;
      for (int k = 0; k < g_.dim; ++k) {
        int64_t bk = pb % Bp;
        pb /= Bp;
        parent_box += (top ? 0 : (bk / 2)) * mul;
        mul *= B;
      }
      int32_t pc = cell_of_box[parent_box];
      if (pc < 0) throw std::runtime_error("planner: parent box without interior");
      prev.cells[ci].parent = pc;
      kids[pc].push_back(int32_t(ci));
    }
  }

  // Groups of level l-1/2 whose survivors are interior here feed the cells.
  std::vector<std::vector<int32_t>> gkids(lev.cells.size());
  if (l > 0) {
    Level& prev = lv_[l - 1];
    for (size_t gi = 0; gi < prev.groups.size(); ++gi) {
      const Group& G = prev.groups[gi];
      const auto& surv = G.skel ? G.sk : G.c;
      if (surv.empty()) continue;
      int64_t d0 = surv[0];
      if (!top && sigma(d0, M) != 0) continue;
      gkids[cell_of_box[top ? 0 : box_of(d0, M)]].push_back(int32_t(gi));
    }
  }

  for (size_t ci = 0; ci < lev.cells.size(); ++ci) {
    Cell& C = lev.cells[ci];
    // Front q^+: surviving fronts of the children that are not interior here,
    // plus active stencil neighbours of the interior.
    std::vector<int32_t> q;
    if (l > 0) {
      for (int32_t k : kids[ci])
        for (int32_t z : lv_[l - 1].cells[k].q)
          if (active_[z] && (top ? false : sigma(z, M) != 0)) q.push_back(z);
    }
    for (int32_t d : C.p)
      for_neighbors(d, [&](int64_t z, int, bool) {
        if (active_[z] && (top ? false : sigma(z, M) != 0)) q.push_back(int32_t(z));
      });
    std::sort(q.begin(), q.end());
    q.erase(std::unique(q.begin(), q.end()), q.end());
    C.q.swap(q);

    // Local numbering [p; q].
    const int32_t np = int32_t(C.p.size());
    for (int32_t i = 0; i < np; ++i) loc_[C.p[i]] = i;
    for (int32_t i = 0; i < int32_t(C.q.size()); ++i) loc_[C.q[i]] = np + i;

    if (l > 0) {
      Level& prev = lv_[l - 1];
      for (int32_t k : kids[ci]) {
        const Cell& K = prev.cells[k];
        Source s;
        s.kind = SRC_CELL_U;
        s.level = l - 1;
        s.index = k;
        s.dim = int32_t(K.q.size());
        s.rowmap = s.colmap = int64_t(lev.maps.size());
        for (int32_t z : K.q) {
          if (active_[z] && loc_[z] < 0)
            throw std::runtime_error("planner: child front unknown lost by its parent");
          lev.maps.push_back(active_[z] ? loc_[z] : -1);
        }
        C.src.push_back(s);
      }
      for (int32_t gi : gkids[ci]) {
        const Group& G = prev.groups[gi];
        const auto& surv = G.skel ? G.sk : G.c;
        Source s;
        s.kind = SRC_GROUP_BASE;
        s.level = l - 1;
        s.index = gi;
        s.dim = int32_t(surv.size());
        s.rowmap = s.colmap = int64_t(lev.maps.size());
        for (int32_t z : surv) {
          if (loc_[z] < 0) throw std::runtime_error("planner: base unknown outside its cell");
          lev.maps.push_back(loc_[z]);
        }
        C.src.push_back(s);
      }
    }
    // Loose stencil entries with an end in p.
    for (int32_t d : C.p) {
      if (!grouped_[d]) C.trips.push_back({loc_[d], loc_[d], int64_t(d)});
      for_neighbors(d, [&](int64_t z, int k, bool up) {
        if (!active_[z]) return;
        if (loc_[z] < 0) throw std::runtime_error("planner: active neighbour outside the front");
        if (grouped_[d] && grouped_[z]) return;
        if (loc_[z] < np && z < d) return;  // interior pair: once
        int64_t lo = up ? d : z;
        C.trips.push_back({loc_[d], loc_[z], link_ref(g_.N, lo, k)});
      });
    }
    for (int32_t d : C.p) loc_[d] = -1;
    for (int32_t d : C.q) loc_[d] = -1;
  }
  // Eliminated unknowns leave the active set.
  for (const Cell& C : lev.cells)
    for (int32_t d : C.p) active_[d] = 0;
  if (top) top_done_ = true;
}

// ---------------------------------------------------------------------------
// Groups of level l+1/2
// ---------------------------------------------------------------------------
void Planner::plan_groups(int l, bool skeletonize) {
  Level& lev = lv_[l];
  lev.groups.clear();
  const int64_t M = g_.m << l;
  (void)skeletonize;

  std::vector<std::pair<int64_t, int32_t>> keyed;
  for (int64_t d = 0; d < g_.N; ++d)
    if (active_[d] && sigma(d, M) == 1) keyed.push_back({group_key(d, M), int32_t(d)});
  std::sort(keyed.begin(), keyed.end());
  std::vector<int32_t> group_of(0);
  for (size_t i = 0; i < keyed.size();) {
    size_t j = i;
    Group G;
    G.gid = keyed[i].first;
    while (j < keyed.size() && keyed[j].first == keyed[i].first) G.c.push_back(keyed[j++].second);
    lev.groups.push_back(std::move(G));
    i = j;
  }
  // Which level-l fronts hold each unknown (at most a few).
  std::vector<int32_t> own0(g_.N, -1), own1(g_.N, -1);
  for (size_t ci = 0; ci < lev.cells.size(); ++ci)
    for (int32_t z : lev.cells[ci].q) {
      if (own0[z] < 0) own0[z] = int32_t(ci);
      else if (own1[z] < 0) own1[z] = int32_t(ci);
      else throw std::runtime_error("planner: unknown in more than two fronts");
    }
  // Earlier bases that land in each group.
  std::vector<int64_t> gkey_index;
  std::vector<std::vector<int32_t>> gkids(lev.groups.size());
  if (l > 0) {
    const Level& prev = lv_[l - 1];
    // map key -> group index
    for (size_t gi = 0; gi < prev.groups.size(); ++gi) {
      const Group& P = prev.groups[gi];
      const auto& surv = P.skel ? P.sk : P.c;
      if (surv.empty()) continue;
      int32_t d0 = surv[0];
      if (sigma(d0, M) != 1) continue;
      int64_t key = group_key(d0, M);
      auto it = std::lower_bound(lev.groups.begin(), lev.groups.end(), key,
                                 [](const Group& a, int64_t k) { return a.gid < k; });
      if (it == lev.groups.end() || it->gid != key)
        throw std::runtime_error("planner: base without group");
      gkids[it - lev.groups.begin()].push_back(int32_t(gi));
    }
  }
  std::vector<uint8_t> in_g(0);
  for (size_t gi = 0; gi < lev.groups.size(); ++gi) {
    Group& G = lev.groups[gi];
    const int32_t nc = int32_t(G.c.size());
    // Neighbour set: the other unknowns of the adjacent fronts and the
    // active stencil neighbours outside c.
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = i;  // mark c
    std::vector<int32_t> cells, cn;
    for (int32_t d : G.c) {
      if (own0[d] >= 0) cells.push_back(own0[d]);
      if (own1[d] >= 0) cells.push_back(own1[d]);
    }
    std::sort(cells.begin(), cells.end());
    cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
    for (int32_t ci : cells)
      for (int32_t z : lev.cells[ci].q)
        if (loc_[z] < 0) cn.push_back(z);
    for (int32_t d : G.c)
      for_neighbors(d, [&](int64_t z, int, bool) {
        if (active_[z] && loc_[z] < 0) cn.push_back(int32_t(z));
      });
    std::sort(cn.begin(), cn.end());
    cn.erase(std::unique(cn.begin(), cn.end()), cn.end());
    G.cN.swap(cn);
    // Rows [c^N; c]: local index of row unknowns; columns: c.
    const int32_t nn = int32_t(G.cN.size());
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = -1;

    // Base formation sources (column side == row side, local in c).
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = i;
    if (l > 0) {
      const Level& prev = lv_[l - 1];
      for (int32_t pg : gkids[gi]) {
        const Group& P = prev.groups[pg];
        const auto& surv = P.skel ? P.sk : P.c;
        Source s;
        s.kind = SRC_GROUP_BASE;
        s.level = l - 1;
        s.index = pg;
        s.dim = int32_t(surv.size());
        s.rowmap = s.colmap = int64_t(lev.maps.size());
        for (int32_t z : surv) {
          if (loc_[z] < 0) throw std::runtime_error("planner: base unknown outside its group");
          lev.maps.push_back(loc_[z]);
        }
        G.bsrc.push_back(s);
      }
    }
    for (int32_t d : G.c) {
      if (!grouped_[d]) G.btrips.push_back({loc_[d], loc_[d], int64_t(d)});
      for_neighbors(d, [&](int64_t z, int k, bool up) {
        if (!active_[z] || loc_[z] < 0 || z < d) return;
        if (grouped_[d] && grouped_[z]) return;
        G.btrips.push_back({loc_[d], loc_[z], link_ref(g_.N, up ? d : z, k)});
      });
    }
    // Loose links between c and c^N (row index in [c^N; c]).
    for (int32_t d : G.c)
      for_neighbors(d, [&](int64_t z, int k, bool up) {
        if (!active_[z] || loc_[z] >= 0) return;
        if (grouped_[d] && grouped_[z]) return;
        auto it = std::lower_bound(G.cN.begin(), G.cN.end(), int32_t(z));
        if (it == G.cN.end() || *it != int32_t(z))
          throw std::runtime_error("planner: stencil neighbour missing from c^N");
        int32_t row = int32_t(it - G.cN.begin());
        G.gtrips.push_back({row, loc_[d], link_ref(g_.N, up ? d : z, k)});
      });
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = -1;

    // Cell update blocks -> [c^N; c] x c.
    for (int32_t i = 0; i < nn; ++i) loc_[G.cN[i]] = i;
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = nn + i;
    for (int32_t ci : cells) {
      const Cell& C = lev.cells[ci];
      Source s;
      s.kind = SRC_CELL_U;
      s.level = l;
      s.index = ci;
      s.dim = int32_t(C.q.size());
      s.rowmap = int64_t(lev.maps.size());
      for (int32_t z : C.q) lev.maps.push_back(loc_[z]);
      s.colmap = int64_t(lev.maps.size());
      for (int32_t z : C.q) lev.maps.push_back(loc_[z] >= nn ? loc_[z] - nn : -1);
      G.gsrc.push_back(s);
    }
    for (int32_t i = 0; i < nn; ++i) loc_[G.cN[i]] = -1;
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = -1;
    G.skel = false;
    G.k = nc;
  }
}

void Planner::set_skeleton(int l, int gi, int k, const int32_t* sk_pos) {
  Group& G = lv_[l].groups.at(gi);
  const int32_t nc = int32_t(G.c.size());
  G.k = k;
  G.sk.clear();
  G.rd.clear();
  G.sk_loc.clear();
  G.rd_loc.clear();
  if (k >= nc) {
    G.skel = false;
    return;
  }
  G.skel = true;
  std::vector<uint8_t> is_sk(nc, 0);
  for (int i = 0; i < k; ++i) is_sk.at(sk_pos[i]) = 1;
  for (int32_t i = 0; i < nc; ++i) {
    if (is_sk[i]) {
      G.sk.push_back(G.c[i]);
      G.sk_loc.push_back(i);
    } else {
      G.rd.push_back(G.c[i]);
      G.rd_loc.push_back(i);
    }
  }
}

void Planner::finish_groups(int l) {
  Level& lev = lv_[l];
  for (Group& G : lev.groups) {
    for (int32_t d : G.c) grouped_[d] = 1;
    if (G.skel)
      for (int32_t d : G.rd) active_[d] = 0;
  }
  lev.groups_done = true;
}

}  // namespace hifde
