// Host-side tree and per-level plans of HIF-DE (Algorithm 4.1).
//
// The planner decides, level by level, which unknowns each cell eliminates
// (Lemma 2.1), which unknowns form each skeletonization group (Lemma 2.4) and
// their neighbour sets c^N, and how every dense block the device builds is
// assembled from blocks of the previous level.  It holds no numerical values:
// the device owns those; the planner only consumes the skeleton choices the
// device's IDs make.
//
// Data flow (multifrontal bookkeeping of the active matrix A_l):
//   * every eliminated cell C leaves an update block U_C on its front q_C
//     (the trailing block of its partially factored frontal matrix);
//   * every group G owns a base block E_G on its current unknowns that holds
//     all entries of A restricted to G not carried by any cell's U;
//   * stencil entries between an unknown that has never been in a group and
//     anything else are "loose": they are read from the stencil when the cell
//     or group that first contains both ends is formed.
// So at level l+1/2, A_{l+1/2}[i,j] = sum_C U_C[i,j] + sum_G E_G[i,j] + loose.
//
// The level-0 cells and the level-1/2 groups depend on the geometry only; a
// tree builds them once (LevelPlan, immutable, shared) and every
// factorization of that tree reuses them.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <vector>

namespace hifde {

struct Geom {
  int dim = 2;
  int64_t n = 0, m = 0, N = 0;
  int L = 0;
  int skip = 0;
  int64_t stride[3] = {1, 1, 1};
};

// Boxes of side m 2^l along an axis (the last one is short when m 2^l does
// not divide n).
inline int64_t boxes_per_axis(const Geom& g, int l) {
  const int64_t M = g.m << l;
  return (g.n + M - 1) / M;
}

// A stencil value: diagonal of unknown d (ref = d) or the link between d and
// d + stride[k] (ref = N * (1 + k) + d).
struct Trip {
  int32_t i, j;
  int64_t ref;
};

enum SrcKind : int32_t {
  SRC_CELL_U = 0,     // trailing (update) block of a cell's frontal matrix
  SRC_GROUP_BASE = 1  // base block of a group
};

struct Source {
  int32_t kind;
  int32_t level;     // integer level l of the cell, or l of group l+1/2
  int32_t index;     // index of the cell/group within its level
  int32_t dim;       // block dimension
  int64_t rowmap;    // offset into the level's map array (dim entries)
  int64_t colmap;    // same, for the column side (== rowmap when symmetric)
};

struct Cell {
  int64_t cid = 0;
  int32_t color = 0;                 // parity of the box coordinates
  std::vector<int32_t> p, q;         // eliminated unknowns, front (sorted)
  std::vector<Source> src;           // extend-add sources
  std::vector<Trip> trips;           // loose stencil entries (local indices)
};

struct Group {
  int64_t gid = 0;
  std::vector<int32_t> c, cN;        // unknowns and neighbour set (sorted)
  std::vector<Source> bsrc;          // base formation: earlier bases
  std::vector<Trip> btrips;          // base formation: loose entries in c
  std::vector<Source> gsrc;          // [c^N; c] x c block: cell update blocks
  std::vector<Trip> gtrips;          // loose links (row in [c^N; c], col in c)
};

// Skeleton choice of a group (value dependent).
struct GroupRes {
  bool skel = false;                 // skeletonized (k < |c|)
  int32_t k = 0;
  std::vector<int32_t> sk, rd;       // skeletons / redundant (sorted, global)
};

// Structure of one level: cells of level l and groups of level l+1/2.
struct LevelPlan {
  std::vector<Cell> cells;
  std::vector<Group> groups;
  std::vector<int32_t> maps;         // maps of the cells' sources
  std::vector<int32_t> gmaps;        // maps of the groups' sources
};

struct Level {
  std::shared_ptr<const LevelPlan> plan;
  std::vector<GroupRes> res;
  const std::vector<Cell>& cells() const { return plan->cells; }
  const std::vector<Group>& groups() const { return plan->groups; }
  const std::vector<int32_t>& survivors(size_t gi) const {
    return res[gi].skel ? res[gi].sk : plan->groups[gi].c;
  }
};

// Per-unknown working arrays of a planner.  A tree keeps them between its
// factorizations, so that a planner does not allocate and first-touch them
// each time; the position maps are all -1 whenever no planning step runs.
struct PlanScratch {
  std::vector<std::vector<int32_t>> loc;
  std::vector<int32_t> own0, own1, act, act_spare;
  std::vector<uint8_t> active, grouped;
  std::vector<uint32_t> geo;    // per unknown, geometry only (see Planner::geo_)
  // the active set once the tree's level-0 cells are eliminated
  std::vector<uint8_t> active0;
  std::vector<int32_t> act0;
};

class Planner {
 public:
  explicit Planner(const Geom& g, std::unique_ptr<PlanScratch> scratch = nullptr);
  // Hands the working arrays back once planning is over (the levels stay).
  std::unique_ptr<PlanScratch> take_scratch();

  const Geom& geom() const { return g_; }
  // Level l cells (l = L gives the top block).  Requires the groups of
  // l-1/2 to be finished.
  void plan_cells(int l);
  // Level l+1/2 groups; requires the cells of level l planned.
  void plan_groups(int l);
  // Record the skeleton choice of group gi of level l+1/2: k skeletons at
  // the given positions of c (sorted ascending).  k >= |c| leaves it alone.
  void set_skeleton(int l, int gi, int k, const int32_t* sk_pos);
  // set_skeleton of every group of level l at once (threaded): group gi has
  // rank ks[gi] and skeleton positions pos[gi * stride ..]
  void set_skeletons(int l, const int32_t* ks, const int32_t* pos, size_t stride);
  // Finish level l+1/2 after every set_skeleton call.
  void finish_groups(int l);

  // The structure of level 0 (cells and groups) as planned so far, to be
  // shared with later factorizations of the same tree.
  std::shared_ptr<const LevelPlan> level0() const { return lv_.at(0).plan; }
  // Start a factorization from a previously planned level 0.
  void adopt_level0(std::shared_ptr<const LevelPlan> p);

  const std::vector<Level>& levels() const { return lv_; }
  const Level& level(int l) const { return lv_.at(l); }

 private:
  int sigma(int64_t d, int l) const;
  void coords(int64_t d, int64_t* x) const;
  int64_t box_of(int64_t d, int l) const;
  int64_t group_key(int64_t d, int l) const;
  template <class F> void for_neighbors(int64_t d, F&& f) const;
  void build_cells(int l, LevelPlan& lp);
  void build_groups(int l, LevelPlan& lp);
  void drop_inactive();
  void fill_act();

  Geom g_;
  std::vector<int8_t> seplev_;       // highest level at which x is a separator
  // per unknown d: byte k (k < 3) = seplev_ of coordinate k (-1 beyond dim);
  // byte 3 bit 2k: x_k > 0, bit 2k+1: x_k < n-1
  std::vector<uint32_t> geo_;
  std::vector<uint8_t> active0_;     // see PlanScratch
  std::vector<int32_t> act0_;
  std::vector<uint8_t> active_, grouped_;
  std::vector<int32_t> act_;         // sorted active unknowns
  std::vector<int32_t> act_spare_;   // drop_inactive's output, swapped with act_
  int32_t* loc(int worker);           // worker's global -> local map (all -1)
  int workers_ = 1;                  // planning threads
  std::vector<std::vector<int32_t>> loc_;
  std::vector<int32_t> own0_, own1_; // scratch: fronts holding an unknown
  std::vector<Level> lv_;
  std::shared_ptr<LevelPlan> building0_;
};

// Frees a planner on a background thread (host memory only).
void discard_planner(std::unique_ptr<Planner> p);
// A factorization's planning starts / ends (discarded planners are freed
// while none is planning).
void planning_begin();
void planning_end();

// f(i) for i in [0, n) on the planner's thread pool, `grain` items at a
// time (the first exception is rethrown).
void plan_parallel(size_t n, size_t grain, const std::function<void(size_t)>& f);

// Validates a tree request; returns an empty string when valid.
std::string check_geom(int dim, int64_t n, int64_t leaf, int skip, Geom* out);

}  // namespace hifde
