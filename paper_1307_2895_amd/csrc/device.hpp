// Descriptors shared by the host orchestration and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hifde {

// A symmetric block read by extend-add: column-major, only its lower
// triangle is valid; it starts at element `off` of pool `pool` of the launch's
// pool table.  rowmap/colmap index the level's map array and give the
// destination row/column of every source index (-1 drops it).
struct SrcDev {
  int64_t off;
  int64_t ld;
  int32_t dim;
  int32_t pool;
  int64_t rowmap;
  int64_t colmap;
};

// Base addresses and element sizes (4: float, 8: double) of the pools the
// sources of one launch refer to.  The pools of one level can differ in
// type: cells eliminated in double beside float groups.
struct PoolTable {
  const void* p[3];
  int32_t esz[3];
};
enum : int32_t { POOL_CELLS = 0, POOL_BASE = 1, POOL_FG = 2 };

// One loose stencil entry: destination (i, j) and the stencil value ref
// (ref < N: diagonal of unknown ref; else offd[ref - N]).
struct TripDev {
  int32_t i, j;
  int64_t ref;
};

// A dense symmetric matrix (column-major, ld = s) in a pool, of which the
// leading p pivots are eliminated by the partial LDL^T.
struct FrontDev {
  int64_t off;
  int32_t s;
  int32_t p;
  int32_t src_begin, src_end;
  int64_t trip_begin, trip_end;
  int64_t idx;      // offset of the front's [p; q] unknown list (solve)
  int32_t color;    // 0/1 checkerboard parity (solve, upward sweep)
  int32_t pad;
};

// A front as the F^-1 sweeps see it: packed apply-form tiles at element
// `off` of the up pool and `offt` of the down (transposed) pool, D^-1 at
// `dv`, unknown list at `idx`.
struct PackDev {
  int64_t off;
  int64_t offt;
  int64_t dv;
  int64_t idx;
  int64_t t_off;     // skeleton fronts: interpolation matrix T (k x p, ld k)
  int64_t cq;        // cells swept in one launch: first row of its x_q update
  int32_t s, p;
};

// Tiles before row tile ti of a packed front with P16 = ceil(p/16) column
// tiles: row tile t holds min(t + 1, P16) tiles.
__host__ __device__ inline int64_t packed_before(int ti, int P16) {
  if (ti <= P16) return int64_t(ti) * (ti + 1) / 2;
  return int64_t(P16) * (P16 + 1) / 2 + int64_t(ti - P16) * P16;
}
__host__ __device__ inline int64_t packed_tiles(int s, int p) {
  return packed_before((s + 15) >> 4, (p + 15) >> 4);
}
// Same for the transposed copy: row tile tc (< ceil(p/16)) holds the
// rt - tc tiles of column tiles tc .. rt - 1.
__host__ __device__ inline int64_t packed_before_t(int tc, int rt) {
  return int64_t(tc) * rt - int64_t(tc) * (tc - 1) / 2;
}

// A skeletonization group.
struct GroupDev {
  int64_t gw_off;    // [c^N; c] x c workspace (ld = nn + nc)
  int64_t base_off;  // base block E_G (nc x nc, lower)
  int64_t fg_off;    // frontal matrix [r; s] x [r; s] (nc x nc)
  int64_t t_off;     // interpolation matrix T (k x r, ld = k)
  int32_t nn, nc;
  int32_t src_begin, src_end;    // cell update blocks feeding the workspace
  int64_t trip_begin, trip_end;  // loose links into the workspace
  int64_t idx;       // offset of the group's unknown list [r; s] (solve)
  int32_t k;         // skeleton count (filled after the ID)
  int32_t skel;      // 1 if skeletonized
};

// A group whose ID runs on a Gaussian sketch Y = Phi M of its block
// M = A_{c^N, c} (rows 0..nn-1 of its workspace, ld nn + nc).
struct SketchDev {
  int64_t m_off;     // M in the group workspace
  int64_t phi_off;   // Phi (r x nn, ld r)
  int64_t y_off;     // Y (r x nc, ld r + nc: the layout of a workspace with r rows)
  int32_t nn, nc, r;
  uint32_t gid;      // the group's key (the generator's counter)
};

}  // namespace hifde
