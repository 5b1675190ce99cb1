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
#pragma once

#include <cstdint>
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

// A stencil value: diagonal of unknown d (ref = d) or the link between d and
// d + stride[k] (ref = N * (1 + k) + d).
struct Trip {
  int32_t i, j;
  int64_t ref;
};

// Where an assembly source lives; resolved to a device pointer by the caller.
enum SrcKind : int32_t {
  SRC_CELL_U = 0,   // trailing (update) block of a cell's frontal matrix
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
  int64_t parent = -1;               // index of the parent cell at level l+1
};

struct Group {
  int64_t gid = 0;
  std::vector<int32_t> c, cN;        // unknowns and neighbour set (sorted)
  std::vector<Source> bsrc;          // base formation: earlier bases
  std::vector<Trip> btrips;          // base formation: loose entries in c
  std::vector<Source> gsrc;          // [c^N; c] x c block: cell update blocks
  std::vector<Trip> gtrips;          // loose links (row in [c^N; c], col in c)
  bool skel = false;                 // skeletonized (0 <= k < |c|)
  int32_t k = 0;
  std::vector<int32_t> sk, rd;       // skeletons / redundant (sorted, global)
  std::vector<int32_t> sk_loc, rd_loc; // same, as positions in c
};

struct Level {
  std::vector<Cell> cells;
  std::vector<Group> groups;
  std::vector<int32_t> maps;         // all maps of this level's sources
  bool groups_done = false;
};

class Planner {
 public:
  Planner(const Geom& g);

  const Geom& geom() const { return g_; }
  // Level l cells (l = L gives the top block).  Requires groups of l-1/2
  // to have their skeletons applied.
  void plan_cells(int l);
  // Level l+1/2 groups; requires cells of level l planned (their interiors
  // are removed from the active set here).
  void plan_groups(int l, bool skeletonize);
  // Record the skeleton choice of group gi of level l+1/2: k skeletons at the
  // given positions of c (sorted ascending).  k == |c| leaves it alone.
  void set_skeleton(int l, int gi, int k, const int32_t* sk_pos);
  // Finish level l+1/2 after every set_skeleton call.
  void finish_groups(int l);

  std::vector<Level>& levels() { return lv_; }
  const std::vector<Level>& levels() const { return lv_; }
  const Cell& top() const { return lv_.back().cells.at(0); }
  bool has_top() const { return top_done_; }
  int64_t active_count() const;

 private:
  int sigma(int64_t d, int64_t M) const;
  void coords(int64_t d, int64_t* x) const;
  bool is_sep(int64_t x, int64_t M) const {
    return ((x + 1) % M == 0) && (x != g_.n - 1);
  }
  int64_t box_of(int64_t d, int64_t M) const;
  int64_t group_key(int64_t d, int64_t M) const;
  template <class F> void for_neighbors(int64_t d, F&& f) const;

  Geom g_;
  std::vector<uint8_t> active_, grouped_;
  std::vector<int32_t> loc_;          // scratch: global -> local (-1)
  std::vector<Level> lv_;
  bool top_done_ = false;
};

// Validates a tree request; returns an empty string when valid.
std::string check_geom(int dim, int64_t n, int64_t leaf, int skip, Geom* out);

}  // namespace hifde
