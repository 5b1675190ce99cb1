// HIF-DE on gfx950: C ABI, factorization driver (Algorithm 4.1), F^-1
// application and preconditioned conjugate gradients.
#include <functional>
#include <future>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/hifde.h"
#include "device.hpp"
#include "planner.hpp"

#include "kernels_factor.inc"
#include "kernels_solve.inc"
#include "kernels_mlp.inc"

namespace hifde {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(x)                                                                  \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      throw ::hifde::Error(e_ == hipErrorOutOfMemory ? HIFDE_ENOMEM : HIFDE_EDEVICE,  \
                           std::string(#x) + ": " + hipGetErrorString(e_));           \
  } while (0)

// Owning device allocation.
struct MemPool;

// A device allocation; with a pool, taken from and given back to it.
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0, cap = 0;         // requested size, size of the block
  MemPool* pool = nullptr;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes), cap(o.cap), pool(o.pool) {
    o.p = nullptr;
    o.bytes = o.cap = 0;
  }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      cap = o.cap;
      pool = o.pool;
      o.p = nullptr;
      o.bytes = o.cap = 0;
    }
    return *this;
  }
  ~DevMem() { release(); }
  inline void release();
  inline void alloc(size_t b);
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Device memory kept for reuse by the factorizations of one tree: blocks that
// a freed factorization gave back are handed out again, best fit among those
// at most twice the request.  Shared by the tree and its factorizations and
// released with the last of them; a failed hipMalloc first releases the kept
// blocks and retries.
struct MemPool {
  std::mutex mu;
  std::multimap<size_t, void*> kept;
  std::atomic<size_t> held{0};    // bytes obtained from hipMalloc, kept or in use
  std::atomic<size_t> limit{0};   // cap on `held` (0: none)
  ~MemPool() { trim(); }
  void* take(size_t b, size_t* cap) {
    {
      std::lock_guard<std::mutex> g(mu);
      auto it = kept.lower_bound(b);
      if (it != kept.end() && it->first / 2 <= b) {
        *cap = it->first;
        void* p = it->second;
        kept.erase(it);
        return p;
      }
    }
    const size_t lim = limit.load();
    if (lim) {
      if (held.load() + b > lim) trim();
      if (held.load() + b > lim)
        throw Error(HIFDE_ENOMEM, "device memory limit of the tree reached (" +
                                      std::to_string(held.load() + b) + " > " +
                                      std::to_string(lim) + " bytes)");
    }
    void* p = nullptr;
    static const bool timing = getenv("HIFDE_TIMING") != nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      trim();
      HIP_CHECK(hipMalloc(&p, b));
    }
    held += b;
    if (timing)
      fprintf(stderr, "[hifde] pool miss: hipMalloc %zu bytes %.3f ms\n", b,
              std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                  .count());
    *cap = b;
    return p;
  }
  void give(void* p, size_t cap) {
    std::lock_guard<std::mutex> g(mu);
    kept.emplace(cap, p);
  }
  void trim() {
    std::lock_guard<std::mutex> g(mu);
    for (auto& kv : kept) {
      (void)hipFree(kv.second);
      held -= kv.first;
    }
    kept.clear();
  }
};

// Streams of freed factorizations, kept for later ones on the same device.
// The first work on a newly created stream has taken milliseconds (its
// binding to a hardware queue), so factorizations take bound streams from
// here and give them back instead of creating and destroying their own.
// They live as long as the process; all have the default priority.
struct StreamCache {
  std::mutex mu;
  std::vector<std::pair<int, hipStream_t>> kept;   // (device, stream)
  static StreamCache& get() {
    static StreamCache* c = new StreamCache;       // never destroyed
    return *c;
  }
  hipStream_t take() {
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    {
      std::lock_guard<std::mutex> g(mu);
      for (size_t i = 0; i < kept.size(); ++i)
        if (kept[i].first == dev) {
          hipStream_t s = kept[i].second;
          kept.erase(kept.begin() + std::ptrdiff_t(i));
          return s;
        }
    }
    hipStream_t s = nullptr;
    HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
  }
  void give(hipStream_t s) {
    if (!s) return;
    hipDevice_t dev = 0;
    if (hipStreamGetDevice(s, &dev) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamDestroy(s);
      return;
    }
    std::lock_guard<std::mutex> g(mu);
    kept.emplace_back(int(dev), s);
  }
};

// Pinned host buffers for the small read-backs of factorizations and
// solves (ranks, pivots, flags, Hessenberg columns).  A copy into pageable
// memory goes through the runtime's staging path, which has been seen to
// start only after work queued earlier on another stream (the side
// stream's apply forms); a copy into pinned memory keeps just its own
// stream's order.  Kept for the life of the process, like the streams.
struct PinnedCache {
  std::mutex mu;
  std::vector<std::pair<void*, size_t>> kept;
  static PinnedCache& get() {
    static PinnedCache* c = new PinnedCache;       // never destroyed
    return *c;
  }
  std::pair<void*, size_t> take() {
    std::lock_guard<std::mutex> g(mu);
    if (kept.empty()) return {nullptr, 0};
    auto b = kept.back();
    kept.pop_back();
    return b;
  }
  void give(void* p, size_t cap) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu);
    kept.emplace_back(p, cap);
  }
};

inline void DevMem::release() {
  if (p) {
    if (pool) pool->give(p, cap);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = cap = 0;
}

inline void DevMem::alloc(size_t b) {
  release();
  if (b == 0) return;
  if (pool) {
    p = pool->take(b, &cap);
  } else {
    HIP_CHECK(hipMalloc(&p, b));
    cap = b;
  }
  bytes = b;
}

// Page-locked host memory (asynchronous device-to-host copies).
struct PinnedMem {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedMem() = default;
  PinnedMem(const PinnedMem&) = delete;
  PinnedMem& operator=(const PinnedMem&) = delete;
  ~PinnedMem() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t b) {
    if (b <= bytes) return;
    release();
    HIP_CHECK(hipHostMalloc(&p, b, hipHostMallocDefault));
    bytes = b;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Bump allocator for the device buffers of one factorization: a few large
// hipMalloc calls instead of one per array, all released together.
// Host-to-device uploads through arenas: count, bytes and host time spent
// in the copy calls (printed per factorization under HIFDE_TIMING).
static std::atomic<int64_t> g_up_n{0}, g_up_bytes{0}, g_up_ns{0};

struct Arena {
  std::vector<DevMem> chunks;
  size_t used = 0;
  MemPool* pool = nullptr;
  static constexpr size_t kChunk = size_t(256) << 20;
  void* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (chunks.empty() || used + bytes > chunks.back().bytes) {
      DevMem m;
      m.pool = pool;
      m.alloc(std::max(bytes, kChunk));
      chunks.push_back(std::move(m));
      used = 0;
    }
    void* p = static_cast<char*>(chunks.back().p) + used;
    used += bytes;
    return p;
  }
  template <class T> T* get(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
  template <class T> T* upload(const std::vector<T>& v, hipStream_t st) {
    T* d = get<T>(std::max<size_t>(1, v.size()));
    if (!v.empty()) {
      const auto t0 = std::chrono::steady_clock::now();
      HIP_CHECK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
      g_up_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(
                     std::chrono::steady_clock::now() - t0).count();
      g_up_n += 1;
      g_up_bytes += int64_t(v.size() * sizeof(T));
    }
    return d;
  }
};

// Packed fronts and work lists of the F^-1 sweeps over one set of fronts:
// the cells of a level (two colors), the skeletonized groups of a level, or
// the top block.  Also the algorithmic work of each launch (for profiling).
struct SweepSet {
  std::vector<PackDev> ph;
  std::vector<int2> up_h[2], down_h;
  std::vector<int2> upf_h[2], downf_h;   // whole-front items (front, 0)
  int64_t pk_elems = 0, pt_elems = 0, dv_elems = 0;
  int kup = 0, kdown = 0;            // rows of x one work-group stages at most
  int kpf = 0;                       // largest 16 ceil(p/16)
  double fac[2] = {0, 0}, srows[2] = {0, 0}, prows[2] = {0, 0};
  PackDev* packs = nullptr;
  int2* up[2] = {nullptr, nullptr};
  int2* down = nullptr;
  int2* upf[2] = {nullptr, nullptr};
  int2* downf = nullptr;
  // upward step of both colors in one launch (cells of level 0): its items,
  // and per distinct q unknown qunk[j] the contribution rows
  // qsrc[qptr[j] .. qptr[j + 1]) that update it, color 0 first
  std::vector<int2> upc_h;
  std::vector<int32_t> qunk_h, qptr_h, qsrc_h;
  int64_t cq_rows = 0;
  int2* upc = nullptr;
  int32_t *qunk = nullptr, *qptr = nullptr, *qsrc = nullptr;
};

// Work lists and per-color work of the fronts in S.ph (colors[i] per front).
static void sweep_items(SweepSet& S, const std::vector<int>& colors) {
  S.up_h[0].clear();
  S.up_h[1].clear();
  S.down_h.clear();
  S.upf_h[0].clear();
  S.upf_h[1].clear();
  S.downf_h.clear();
  S.kup = S.kdown = S.kpf = 0;
  for (int c = 0; c < 2; ++c) S.fac[c] = S.srows[c] = S.prows[c] = 0;
  for (size_t fi = 0; fi < S.ph.size(); ++fi) {
    const PackDev& f = S.ph[fi];
    const int c = colors[fi];
    const int rt = (f.s + 15) >> 4, P16 = (f.p + 15) >> 4;
    for (int t = 0; t < rt; t += kSwWaves) {
      S.up_h[c].push_back(make_int2(int(fi), t));
      S.kup = std::max(S.kup, std::min(f.p, 16 * std::min(P16, std::min(rt, t + kSwWaves))));
    }
    for (int t = 0; t < P16; t += kSwWaves) S.down_h.push_back(make_int2(int(fi), t));
    S.kdown = std::max(S.kdown, 16 * rt);
    if (P16 > 0) {
      S.upf_h[c].push_back(make_int2(int(fi), 0));
      S.downf_h.push_back(make_int2(int(fi), 0));
      S.kpf = std::max(S.kpf, 16 * P16);
    }
    S.fac[c] += 0.5 * double(f.p) * (f.p + 1) + double(f.s - f.p) * f.p;
    S.srows[c] += f.s;
    S.prows[c] += f.p;
  }
}

// Packed layout of the fronts fh, back to back; with `worst`, every front
// gets the slots of p = s (its pivot count is not known yet).
static void sweep_layout(SweepSet& S, const std::vector<FrontDev>& fh, bool worst) {
  S = SweepSet{};
  for (const FrontDev& f : fh) {
    PackDev q{};
    q.off = S.pk_elems;
    q.offt = S.pt_elems;
    q.dv = S.dv_elems;
    q.idx = f.idx;
    q.s = f.s;
    q.p = f.p;
    const int pc = worst ? f.s : f.p;
    S.pk_elems += packed_tiles(f.s, pc) * 256;
    S.pt_elems += packed_tiles(f.s, pc) * 256;
    S.dv_elems += pc;
    S.ph.push_back(q);
  }
}

// Rows of the contribution buffer for the one-launch upward step of
// colored fronts: front f (with pivots) owns rows f.cq .. f.cq + s - p - 1,
// and each distinct q unknown gets the rows that update it, color 0 first
// (a counting sort by unknown; N unknowns).  Left empty when two fronts of
// one color share a q unknown (the colored launches would race there).
static void contrib_plan(SweepSet& S, const std::vector<int32_t>& idx_h,
                         const std::vector<int>& colors, int64_t N) {
  int64_t rows = 0;
  std::vector<int32_t> start(size_t(N) + 1, 0);
  for (PackDev& f : S.ph) {
    if (f.p == 0) continue;
    f.cq = rows;
    rows += f.s - f.p;
    for (int i = f.p; i < f.s; ++i) ++start[size_t(idx_h[size_t(f.idx) + i]) + 1];
  }
  if (rows == 0 || rows > INT32_MAX) return;
  for (int64_t u = 0; u < N; ++u) start[size_t(u) + 1] += start[size_t(u)];
  std::vector<int32_t> fill(start.begin(), start.end() - 1);
  std::vector<int32_t> src(static_cast<size_t>(rows));
  std::vector<int8_t> col(static_cast<size_t>(rows));
  for (int c = 0; c < 2; ++c)
    for (size_t fi = 0; fi < S.ph.size(); ++fi) {
      const PackDev& f = S.ph[fi];
      if (f.p == 0 || colors[fi] != c) continue;
      for (int i = f.p; i < f.s; ++i) {
        const int32_t k = fill[size_t(idx_h[size_t(f.idx) + i])]++;
        src[size_t(k)] = int32_t(f.cq + i - f.p);
        col[size_t(k)] = int8_t(c);
      }
    }
  std::vector<int32_t> qunk, qptr{0};
  for (int64_t u = 0; u < N; ++u) {
    const int32_t a = start[size_t(u)], b = start[size_t(u) + 1];
    if (a == b) continue;
    for (int32_t k = a + 1; k < b; ++k)
      if (col[size_t(k)] <= col[size_t(k) - 1]) return;
    qunk.push_back(int32_t(u));
    qptr.push_back(b);
  }
  for (size_t fi = 0; fi < S.ph.size(); ++fi)
    if (S.ph[fi].p > 0) S.upc_h.push_back(make_int2(int(fi), 0));
  S.qunk_h = std::move(qunk);
  S.qptr_h = std::move(qptr);
  S.qsrc_h = std::move(src);
  S.cq_rows = rows;
}

// contrib_n > 0: also plan the one-launch upward step (contrib_n unknowns).
static void build_sweep(SweepSet& S, const std::vector<FrontDev>& fh, bool colored,
                        const std::vector<int32_t>* idx_h = nullptr, int64_t contrib_n = 0) {
  sweep_layout(S, fh, false);
  std::vector<int> colors(fh.size(), 0);
  if (colored)
    for (size_t i = 0; i < fh.size(); ++i) colors[i] = fh[i].color & 1;
  sweep_items(S, colors);
  if (idx_h && contrib_n > 0) contrib_plan(S, *idx_h, colors, contrib_n);
}

static void upload_sweep(SweepSet& S, Arena& mem, hipStream_t st) {
  S.packs = mem.upload(S.ph, st);
  S.up[0] = mem.upload(S.up_h[0], st);
  S.up[1] = mem.upload(S.up_h[1], st);
  S.down = mem.upload(S.down_h, st);
  S.upf[0] = mem.upload(S.upf_h[0], st);
  S.upf[1] = mem.upload(S.upf_h[1], st);
  S.downf = mem.upload(S.downf_h, st);
  if (!S.upc_h.empty()) {
    S.upc = mem.upload(S.upc_h, st);
    S.qunk = mem.upload(S.qunk_h, st);
    S.qptr = mem.upload(S.qptr_h, st);
    S.qsrc = mem.upload(S.qsrc_h, st);
  }
}

// Device description of the cells of one level; depends on the plan only, so
// the level-0 one is shared by every factorization of a tree.
struct CellStatic {
  std::vector<FrontDev> fh;
  std::vector<SrcDev> srcs_h;
  std::vector<TripDev> trips_h;
  std::vector<int32_t> idx_h;
  // per front row (laid out like idx): the first column of the assembled
  // front's lower triangle that row has a nonzero in.  Elimination fills
  // only to the right of it (the envelope), so an update whose panel
  // columns all lie left of every envelope start of a tile's rows (or of
  // its columns) adds exact zeros there and is skipped.
  std::vector<int32_t> env_h;
  // widest band of the eliminated blocks: max over p rows i of i - env(i)
  int pband = 0;
  const std::vector<int32_t>* maps_h = nullptr;
  Arena mem;
  FrontDev* fronts = nullptr;
  SrcDev* srcs = nullptr;
  int32_t* maps = nullptr;
  TripDev* trips = nullptr;
  int32_t* idx = nullptr;
  int32_t* env = nullptr;
  int64_t elems = 0;
  int pmax = 0, smax = 0, ncell = 0;
  bool on_device = false;
  SweepSet sw;                       // F^-1 sweeps (two colors)
};

// Device description of the groups of one level (before the IDs).
struct GroupStatic {
  std::vector<GroupDev> gh;          // gw/base/t offsets, sizes, source ranges
  std::vector<FrontDev> bf;          // base-formation "fronts"
  std::vector<SrcDev> bsrcs_h, gsrcs_h;
  std::vector<TripDev> btrips_h, gtrips_h;
  const std::vector<int32_t>* maps_h = nullptr;
  Arena mem;
  FrontDev* bfronts = nullptr;
  int32_t* maps = nullptr;
  SrcDev* bsrcs = nullptr;
  SrcDev* gsrcs = nullptr;
  TripDev* btrips = nullptr;
  TripDev* gtrips = nullptr;
  int64_t base_elems = 0, gw_elems = 0, t_elems = 0;
  int ncmax = 0;
  bool on_device = false;
};

// Per-factorization state of one level.
struct CellLevel {
  std::shared_ptr<CellStatic> st;
  void* pool = nullptr;              // frontal matrices
  int esz = 0;                       // their element size (4 or 8)
  int* info = nullptr;
  void *pk = nullptr, *pt = nullptr, *dinv = nullptr;  // packed apply form (up, down), D^-1
};

struct GroupLevel {
  std::shared_ptr<GroupStatic> st;
  int esz = 0;                       // element size of base, gather, T and fronts
  std::vector<GroupDev> gh;          // with k, skel, fg_off, idx filled in
  GroupDev* groups = nullptr;
  void *base = nullptr, *gw = nullptr, *fg = nullptr, *tpool = nullptr;
  int32_t *kout = nullptr, *perm = nullptr, *gsel = nullptr, *idx = nullptr;
  FrontDev* fgfronts = nullptr;
  int* info = nullptr;
  std::vector<FrontDev> ff;
  std::vector<int32_t> gsel_h, idx_h;
  int64_t perm_stride = 0;
  int nskel = 0, ngroup = 0, ncskel = 0;
  SweepSet sw;                       // F^-1 sweeps over the skeleton fronts
  void *pk = nullptr, *pt = nullptr, *dinv = nullptr;
  // interpolation work: elements kr, rows r and k
  double tel = 0, rrows = 0, krows = 0;
  // predicted ranks (model) and the event that makes them readable
  int32_t* khat_d = nullptr;
  std::shared_ptr<PinnedMem> khat_h;
  hipEvent_t pred_ev = nullptr;
};

}  // namespace hifde

using namespace hifde;

struct hifde_tree_s {
  std::shared_ptr<MemPool> pool = std::make_shared<MemPool>();   // factorizations' memory
  std::mutex scratch_mu;                                         // planners' working arrays
  std::vector<std::unique_ptr<PlanScratch>> scratch;
  std::unique_ptr<PlanScratch> take_scratch() {
    std::lock_guard<std::mutex> g(scratch_mu);
    if (scratch.empty()) return nullptr;
    auto s = std::move(scratch.back());
    scratch.pop_back();
    return s;
  }
  void give_scratch(std::unique_ptr<PlanScratch> s) {
    std::lock_guard<std::mutex> g(scratch_mu);
    scratch.push_back(std::move(s));
  }
  Geom g;
  std::map<uint64_t, int> tune;             // autotuner choices (see tune_choice)
  std::vector<float> model;                 // rank predictor weights (host)
  DevMem model_d;                           // and on the device
  std::shared_ptr<const LevelPlan> l0;      // level-0 cells and level-1/2 groups
  std::shared_ptr<CellStatic> c0;           // their device descriptions
  std::shared_ptr<GroupStatic> g0;
  size_t c0_esz = 0;
};

struct hifde_factor_s {
  // declared first: released after every member that allocated from it
  std::shared_ptr<MemPool> pool;
  Geom g;
  hifde_precision prec = HIFDE_FP64;
  double eps = 0.0;
  bool definite = true;        // without HIFDE_INDEFINITE: pivots must be positive
  bool sketch = false;         // HIFDE_SKETCH_ID
  bool plan_only = false;
  std::unique_ptr<Planner> planner;
  std::vector<CellLevel> cl;   // L + 1 entries (last = top)
  std::vector<GroupLevel> gl;  // L entries
  Arena mem;
  DevMem diag, offd;
  hifde_stats_t stats{};
  // solver scratch (C: x_q contributions of the one-launch upward step)
  DevMem X, Z, C;
  DevMem pcg;
  int64_t pcg_rhs = 0;
  DevMem gm;                   // GMRES basis, kept z_k and scalars
  // kernel timing (hifde_profile)
  struct ProfEvent {
    hipEvent_t a = nullptr, b = nullptr;
    int cls = 0;
    double bytes = 0, flops = 0;
  };
  uint32_t prof_mask = 0;
  int prof_level = -1;
  std::vector<ProfEvent> prof_ev;
  size_t prof_used = 0;
  hifde_prof_t prof_acc[HIFDE_PROF_CLASSES]{};
  // skeleton-front launches before the IDs return: 0 = after (exact
  // sizes), 1 = bounded by the rank model's predictions, 2 = worst case
  int presize = 0;
  hipStream_t aux = nullptr;               // rank-model inference
  hipStream_t side = nullptr;              // apply forms and packing of the cells
  hipEvent_t offd_ev = nullptr;            // stencil ready (for aux)
  const float* model = nullptr;            // device weights (tree-owned)
  std::vector<hipEvent_t> events;          // created here, destroyed with F
  int64_t rank_groups = 0, skel_panels = 0, rebuckets = 0;
  bool autotune = false;                   // HIFDE_AUTOTUNE
  hifde_tree_s* tree = nullptr;            // owner of the tuning cache
  int64_t tuned = 0;
  double rank_abs_err = 0;
  // captured F^-1 application (one per right-hand-side count and buffers)
  bool use_graph = true;
  bool row_tiles = false;                  // HIFDE_SWEEP_ROW_TILES
  int* bad_d = nullptr;                    // k_stencil's input flags
  // Pinned buffer of at least n bytes for a read-back.  Every read-back
  // synchronizes its stream before the next one asks, so the buffer is
  // never replaced under a copy in flight.
  void* hs = nullptr;
  size_t hs_cap = 0;
  void* host_stage(size_t n) {
    if (!hs) {
      auto b = PinnedCache::get().take();
      hs = b.first;
      hs_cap = b.second;
    }
    if (n > hs_cap) {
      if (hs) HIP_CHECK(hipHostFree(hs));
      hs = nullptr;
      hs_cap = 0;
      const size_t c = std::max<size_t>(n, size_t(1) << 20);
      HIP_CHECK(hipHostMalloc(&hs, c, hipHostMallocDefault));
      hs_cap = c;
    }
    return hs;
  }
  bool input_checked = false;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_nrhs = 0;
  const void *g_x = nullptr, *g_z = nullptr, *g_c = nullptr;
  int g_part = 0;
  // one-launch level-0 upward step: 0 both kernels, 1 the sweep only, 2 the
  // contribution add only (a timed sweep launched apart from the graph)
  int upc_part = 0;
  // The side stream, after the work queued on st so far.
  hipStream_t side_after(hipStream_t st) {
    if (!side) side = StreamCache::get().take();
    hipEvent_t e = new_event();
    HIP_CHECK(hipEventRecord(e, st));
    HIP_CHECK(hipStreamWaitEvent(side, e, 0));
    return side;
  }
  // Apply form and packing of the last cell level: queued on the side
  // stream once that level's IDs are launched, so that they do not compete
  // with the IDs, whose ranks the host waits for.
  std::function<void(hipStream_t)> side_work;
  void flush_side(hipStream_t st) {
    if (!side_work) return;
    std::function<void(hipStream_t)> w = std::move(side_work);
    side_work = nullptr;
    w(side_after(st));
  }
  // Later work on st waits for the side stream's.
  void join_side(hipStream_t st) {
    if (!side) return;
    hipEvent_t e = new_event();
    HIP_CHECK(hipEventRecord(e, side));
    HIP_CHECK(hipStreamWaitEvent(st, e, 0));
  }
  hipEvent_t new_event() {
    hipEvent_t e = nullptr;
    HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    events.push_back(e);
    return e;
  }
  void use_pool(std::shared_ptr<MemPool> p) {
    pool = std::move(p);
    for (DevMem* m : {&diag, &offd, &X, &Z, &C, &pcg, &gm}) m->pool = pool.get();
    mem.pool = pool.get();
  }
  // Releases the runtime handles (idempotent).
  void release_handles() {
    if (skel_job.valid()) {   // (a failure elsewhere: its own error is moot)
      try {
        skel_job.get();
      } catch (...) {
      }
    }
    // blocks go back to the pool for reuse: no kernel may still use them
    if (pool) (void)hipDeviceSynchronize();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    events.clear();
    StreamCache::get().give(aux);
    aux = nullptr;
    StreamCache::get().give(side);
    side = nullptr;
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    StreamCache::get().give(cap);
    cap = nullptr;
    PinnedCache::get().give(hs, hs_cap);
    hs = nullptr;
    hs_cap = 0;
    for (ProfEvent& e : prof_ev) {
      if (e.a) (void)hipEventDestroy(e.a);
      if (e.b) (void)hipEventDestroy(e.b);
    }
    prof_ev.clear();
  }
  // A level's skeleton fronts, prepared and launched on a helper thread
  // while the host plans the next level (join_skel before the arena, the
  // stream or that level's descriptors are used again).
  std::future<void> skel_job;
  void join_skel() {
    if (skel_job.valid()) skel_job.get();
  }
  ~hifde_factor_s() { release_handles(); }
};

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <class Fn> static int guarded(Fn&& fn) {
  try {
    fn();
    return HIFDE_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(HIFDE_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(HIFDE_EINVAL, e.what());
  }
}

namespace hifde {

static inline unsigned nblk(int64_t n, int t = kThreads) { return unsigned((n + t - 1) / t); }

// Host-side phase timer, printed to stderr when HIFDE_TIMING is set.
struct PhaseTimer {
  bool on = getenv("HIFDE_TIMING") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char* what, int l) {
    if (!on) return;
    auto now = std::chrono::steady_clock::now();
    fprintf(stderr, "[hifde] level %d %-18s %8.3f ms\n", l, what,
            std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

// ---------------------------------------------------------------------------
// Source resolution: pool and element offset of a planned block.
// ---------------------------------------------------------------------------
static SrcDev resolve(const hifde_factor_s& F, const Source& s) {
  SrcDev d{};
  d.dim = s.dim;
  d.rowmap = s.rowmap;
  d.colmap = s.colmap;
  if (s.kind == SRC_CELL_U) {
    const FrontDev& f = F.cl.at(s.level).st->fh.at(s.index);
    d.pool = POOL_CELLS;
    d.off = f.off + f.p + int64_t(f.p) * f.s;
    d.ld = f.s;
  } else {
    const GroupDev& g = F.gl.at(s.level).gh.at(s.index);
    if (g.skel) {
      const int r = g.nc - g.k;
      d.pool = POOL_FG;
      d.off = g.fg_off + r + int64_t(r) * g.nc;
    } else {
      d.pool = POOL_BASE;
      d.off = g.base_off;
    }
    d.ld = g.nc;
  }
  return d;
}

// `one_launch`: also plan the upward step of both colors in one launch.
static std::shared_ptr<CellStatic> make_cell_static(const hifde_factor_s& F, const LevelPlan& lp,
                                                    bool one_launch) {
  auto cs = std::make_shared<CellStatic>();
  const size_t nc = lp.cells.size();
  // offsets first (in order), then every cell's lists in parallel
  cs->fh.resize(nc);
  int64_t off = 0, nsrc = 0, ntrip = 0, nidx = 0;
  for (size_t ci = 0; ci < nc; ++ci) {
    const Cell& c = lp.cells[ci];
    FrontDev& f = cs->fh[ci];
    f = FrontDev{};
    f.off = off;
    f.p = int32_t(c.p.size());
    f.s = int32_t(c.p.size() + c.q.size());
    f.src_begin = int32_t(nsrc);
    nsrc += int64_t(c.src.size());
    f.src_end = int32_t(nsrc);
    f.trip_begin = ntrip;
    ntrip += int64_t(c.trips.size());
    f.trip_end = ntrip;
    f.idx = nidx;
    nidx += f.s;
    f.color = c.color;
    off += int64_t(f.s) * f.s;
    cs->pmax = std::max(cs->pmax, f.p);
    cs->smax = std::max(cs->smax, f.s);
  }
  cs->srcs_h.resize(size_t(nsrc));
  cs->trips_h.resize(size_t(ntrip));
  cs->idx_h.resize(size_t(nidx));
  cs->env_h.resize(size_t(nidx));
  std::vector<int32_t> band(nc, 0);
  plan_parallel(nc, 16, [&](size_t ci) {
    const Cell& c = lp.cells[ci];
    const FrontDev& f = cs->fh[ci];
    for (size_t k = 0; k < c.src.size(); ++k) cs->srcs_h[size_t(f.src_begin) + k] = resolve(F, c.src[k]);
    int32_t* env = cs->env_h.data() + f.idx;
    for (int32_t i = 0; i < f.s; ++i) env[i] = i;
    for (size_t k = 0; k < c.trips.size(); ++k) {
      const Trip& t = c.trips[k];
      cs->trips_h[size_t(f.trip_begin) + k] = TripDev{t.i, t.j, t.ref};
      const int32_t hi = std::max(t.i, t.j), lo = std::min(t.i, t.j);
      env[hi] = std::min(env[hi], lo);
    }
    // a source block is dense: each row it reaches has a nonzero in the
    // source's first destination column
    for (const Source& src : c.src) {
      const int32_t* m = lp.maps.data() + src.rowmap;
      int32_t mn = f.s;
      for (int32_t a = 0; a < src.dim; ++a)
        if (m[a] >= 0) mn = std::min(mn, m[a]);
      for (int32_t a = 0; a < src.dim; ++a)
        if (m[a] >= 0) env[m[a]] = std::min(env[m[a]], mn);
    }
    for (int32_t i = 0; i < f.p; ++i) band[ci] = std::max(band[ci], i - env[i]);
    std::copy(c.p.begin(), c.p.end(), cs->idx_h.begin() + f.idx);
    std::copy(c.q.begin(), c.q.end(), cs->idx_h.begin() + f.idx + int64_t(c.p.size()));
  });
  cs->elems = off;
  for (int32_t b : band) cs->pband = std::max(cs->pband, int(b));
  cs->ncell = int(cs->fh.size());
  cs->maps_h = &lp.maps;
  build_sweep(cs->sw, cs->fh, true, &cs->idx_h, one_launch ? F.g.N : 0);
  return cs;
}

// Device copies of the descriptors, in `mem` (the tree-shared level-0
// descriptors keep their own arena; later levels use the factor's).
static void upload_cell_static(CellStatic& cs, Arena& mem, hipStream_t st) {
  if (cs.on_device) return;
  cs.fronts = mem.upload(cs.fh, st);
  cs.srcs = mem.upload(cs.srcs_h, st);
  cs.maps = mem.upload(*cs.maps_h, st);
  cs.trips = mem.upload(cs.trips_h, st);
  cs.idx = mem.upload(cs.idx_h, st);
  cs.env = mem.upload(cs.env_h, st);
  upload_sweep(cs.sw, mem, st);
  cs.on_device = true;
}

static std::shared_ptr<GroupStatic> make_group_static(const hifde_factor_s& F,
                                                      const LevelPlan& lp, bool skel) {
  auto gs = std::make_shared<GroupStatic>();
  const size_t ng = lp.groups.size();
  // offsets first (in order), then every group's lists in parallel
  gs->gh.resize(ng);
  gs->bf.resize(ng);
  int64_t base_off = 0, gw_off = 0, t_off = 0, nbs = 0, nbt = 0, ngs = 0, ngt = 0;
  for (size_t gi = 0; gi < ng; ++gi) {
    const Group& g = lp.groups[gi];
    GroupDev& d = gs->gh[gi];
    d = GroupDev{};
    d.nc = int32_t(g.c.size());
    d.nn = int32_t(g.cN.size());
    d.base_off = base_off;
    d.gw_off = gw_off;
    d.t_off = t_off;
    FrontDev& f = gs->bf[gi];
    f = FrontDev{};
    f.off = base_off;
    f.s = d.nc;
    f.p = 0;
    f.src_begin = int32_t(nbs);
    nbs += int64_t(g.bsrc.size());
    f.src_end = int32_t(nbs);
    f.trip_begin = nbt;
    nbt += int64_t(g.btrips.size());
    f.trip_end = nbt;
    d.src_begin = int32_t(ngs);
    ngs += int64_t(g.gsrc.size());
    d.src_end = int32_t(ngs);
    d.trip_begin = ngt;
    ngt += int64_t(g.gtrips.size());
    d.trip_end = ngt;
    base_off += int64_t(d.nc) * d.nc;
    if (skel) {
      gw_off += (int64_t(d.nn) + d.nc) * d.nc;
      t_off += int64_t(d.nc) * d.nc / 4 + 1;  // k (n-k) <= n^2/4
    }
    gs->ncmax = std::max(gs->ncmax, int(d.nc));
  }
  gs->bsrcs_h.resize(size_t(nbs));
  gs->btrips_h.resize(size_t(nbt));
  gs->gsrcs_h.resize(size_t(ngs));
  gs->gtrips_h.resize(size_t(ngt));
  plan_parallel(ng, 16, [&](size_t gi) {
    const Group& g = lp.groups[gi];
    const GroupDev& d = gs->gh[gi];
    const FrontDev& f = gs->bf[gi];
    for (size_t k = 0; k < g.bsrc.size(); ++k)
      gs->bsrcs_h[size_t(f.src_begin) + k] = resolve(F, g.bsrc[k]);
    for (size_t k = 0; k < g.btrips.size(); ++k) {
      const Trip& t = g.btrips[k];
      gs->btrips_h[size_t(f.trip_begin) + k] = TripDev{t.i, t.j, t.ref};
    }
    for (size_t k = 0; k < g.gsrc.size(); ++k)
      gs->gsrcs_h[size_t(d.src_begin) + k] = resolve(F, g.gsrc[k]);
    for (size_t k = 0; k < g.gtrips.size(); ++k) {
      const Trip& t = g.gtrips[k];
      gs->gtrips_h[size_t(d.trip_begin) + k] = TripDev{t.i, t.j, t.ref};
    }
  });
  gs->base_elems = base_off;
  gs->gw_elems = gw_off;
  gs->t_elems = t_off;
  gs->maps_h = &lp.gmaps;
  return gs;
}

static void upload_group_static(GroupStatic& gs, Arena& mem, hipStream_t st) {
  if (gs.on_device) return;
  gs.bfronts = mem.upload(gs.bf, st);
  gs.maps = mem.upload(*gs.maps_h, st);
  gs.bsrcs = mem.upload(gs.bsrcs_h, st);
  gs.btrips = mem.upload(gs.btrips_h, st);
  gs.gsrcs = mem.upload(gs.gsrcs_h, st);
  gs.gtrips = mem.upload(gs.gtrips_h, st);
  gs.on_device = true;
}

// Grid of a front_tile launch: nf fronts, nt tiles each.
static unsigned front_tile_grid(unsigned nf, int64_t nt, const char* what) {
  const int64_t per = nf >= 8 ? 0 : 8 / front_tile_round(int(nf));
  const int64_t g = nf >= 8 ? int64_t(8) * ((nf + 7) / 8) * nt : int64_t(8) * ((nt + per - 1) / per);
  if (g > INT32_MAX) throw Error(HIFDE_EINVAL, std::string("front too large for the ") + what);
  return unsigned(g);
}

// Batched partial LDL^T of a set of fronts already in `pool`.
// Fronts with more than j pivots: all of them, or (fh sorted by p,
// descending) the leading ones only.
static unsigned active_fronts(const std::vector<FrontDev>& fh, int j, bool sorted) {
  if (!sorted) return unsigned(fh.size());
  unsigned n = 0;
  while (n < fh.size() && fh[n].p > j) ++n;
  return n;
}

// Trailing-update variants of the batched LDL^T.
// LDL_MFMA takes the panels in pairs (one pass of the trailing block per
// two panels); LDL_MFMA1 one at a time, whose narrower panels skip more
// tiles outside the fronts' envelopes.
// LDL_BAND eliminates banded cells in one launch (k_ldl_band), when the
// level's band is narrower than a panel.
enum { LDL_FMA = 0, LDL_MFMA = 1, LDL_FRONT = 2, LDL_MFMA1 = 3, LDL_BAND = 4, LDL_VARIANTS = 5 };
// Variants the tuner times for a launch of nf fronts: the one-launch form
// (one work-group per front) and the single-panel matrix-core form only
// when the fronts fill the device.
static inline int ldl_timed(int64_t nf) { return nf >= 256 ? LDL_VARIANTS : LDL_FRONT; }

// With `bounds`, the p of fh are upper bounds of the device fronts' pivot
// counts (the device holds the exact ones); launch shapes then cover any
// count up to the bound.  With `sorted` (fh by p, descending), the launches
// of panel j cover only the fronts that still have pivots there.
template <typename T>
static void batched_ldl(T* pool, const std::vector<FrontDev>& fh, const FrontDev* fronts_d,
                        int* info_d, int definite, hipStream_t st, bool bounds = false,
                        bool sorted = false, int variant = LDL_MFMA, int* counter = nullptr,
                        const int32_t* env = nullptr, int band = -1) {
  if (fh.empty()) return;
  if (variant == LDL_BAND) {
    int pm = 0;
    for (const auto& f : fh) pm = std::max(pm, f.p);
    const int bwt = band < 8 ? 8 : band < 16 ? 16 : band < 17 ? 17 : 32;
    const size_t smem = (size_t(bwt * bwt) +
                         size_t(std::max((pm + bwt) * bwt, 2 * kTB * (kNB + 1))) + size_t(2 * pm)) *
                        sizeof(T);
    if (!bounds && band >= 0 && band < kNB && smem <= 64 * 1024) {
      const dim3 g(unsigned(fh.size()));
      if (band < 8)
        hipLaunchKernelGGL((k_ldl_band<T, 8>), g, dim3(kThreads), smem, st, pool, fronts_d,
                           info_d, definite, band);
      else if (band < 16)
        hipLaunchKernelGGL((k_ldl_band<T, 16>), g, dim3(kThreads), smem, st, pool, fronts_d,
                           info_d, definite, band);
      else if (band < 17)
        hipLaunchKernelGGL((k_ldl_band<T, 17>), g, dim3(kThreads), smem, st, pool, fronts_d,
                           info_d, definite, band);
      else
        hipLaunchKernelGGL((k_ldl_band<T, 32>), g, dim3(kThreads), smem, st, pool, fronts_d,
                           info_d, definite, band);
      HIP_CHECK(hipGetLastError());
      return;
    }
    variant = LDL_MFMA;
  }
  if (variant == LDL_FRONT && counter) {
    // one persistent launch: a full round of the device, fronts from a queue
    static const std::pair<int, int> occ = [] {
      int dev = 0, cus = 0, per_cu = 0;
      HIP_CHECK(hipGetDevice(&dev));
      HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&k_ldl_front<T>), kThreads, 0));
      return std::make_pair(per_cu, cus);
    }();
    const int per_cu = occ.first, cus = occ.second;
    const int64_t nf = int64_t(fh.size());
    const unsigned grid =
        unsigned(std::max<int64_t>(1, std::min<int64_t>(nf, int64_t(std::max(1, per_cu)) *
                                                                std::max(1, cus))));
    HIP_CHECK(hipMemsetAsync(counter, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_ldl_front<T>, dim3(grid), dim3(kThreads), 0, st, pool, fronts_d, int(nf),
                       info_d, definite, counter);
    HIP_CHECK(hipGetLastError());
    return;
  }
  if (variant == LDL_FRONT) variant = LDL_MFMA;
  int pmax = 0;
  for (const auto& f : fh) pmax = std::max(pmax, f.p);
  // Tiles of an update whose trailing block starts `w` columns after j0
  // (w(f) = columns applied); `first_col`: the first tile column only.
  auto tiles = [&](int j0, int width, bool first_col) {
    int64_t mt = 0;
    for (const auto& f : fh) {
      if (j0 >= f.p) continue;
      const int r0 = bounds ? j0 + 1 : j0 + std::min(width, f.p - j0);
      const int64_t nt = f.s - r0;
      if (nt <= 0) continue;
      const int64_t T_ = (nt + kTB - 1) / kTB;
      mt = std::max(mt, first_col ? T_ : T_ * (T_ + 1) / 2);
    }
    return mt;
  };
  auto panel = [&](int j0) {   // diagonal block and rows of panel j0
    const unsigned nf = active_fronts(fh, j0, sorted);
    int64_t maxr = 0;
    for (const auto& f : fh) {
      if (j0 >= f.p) continue;
      const int r0 = bounds ? j0 + 1 : std::min(j0 + kNB, f.p);
      if (f.s > r0) maxr = std::max<int64_t>(maxr, (f.s - r0 + 63) / 64);
    }
    // one wavefront per diagonal block: the 32 dependent steps are latency
    // bound, so many small work-groups per CU do better than few large ones
    hipLaunchKernelGGL(k_ldl_diag<T>, dim3(nf), dim3(kDiagThreads), 0, st, pool, fronts_d, j0,
                       info_d, definite);
    // (rows of exact zeros are skipped only where every pivot is positive:
    // an indefinite pivot would turn their zeros into -0)
    if (maxr > 0)
      hipLaunchKernelGGL(k_ldl_rows<T>, dim3(front_tile_grid(nf, maxr, "panel grid")),
                         dim3(kThreads), 0, st, pool, fronts_d, j0, int(nf), int(maxr),
                         definite ? env : nullptr);
  };
  auto update = [&](unsigned nf, int j0, int64_t mt, int mode) {
    if (mt <= 0) return;
    const unsigned g = front_tile_grid(nf, mt, "trailing-update grid");
    if (variant == LDL_MFMA || variant == LDL_MFMA1)
      hipLaunchKernelGGL(k_ldl_update_mfma<T>, dim3(g), dim3(kThreads), 0, st, pool, fronts_d,
                         j0, int(nf), int(mt), mode, env);
    else
      hipLaunchKernelGGL(k_ldl_update<T>, dim3(g), dim3(kThreads), 0, st, pool, fronts_d, j0,
                         int(nf), int(mt), env);
  };
  // panels in pairs (delayed update) on the matrix cores, one at a time
  // otherwise.  Pairs start at multiples of 2 kNB whatever the counts (a
  // pair without its second panel sums as a single update), so bounded and
  // exact pivot counts give the same arithmetic.
  const bool pairs = variant == LDL_MFMA;
  for (int j0 = 0; j0 < pmax;) {
    const unsigned nf = active_fronts(fh, j0, sorted);
    if (nf == 0) break;
    panel(j0);
    const bool next = pairs && j0 + kNB < pmax;
    if (!next) {
      update(nf, j0, tiles(j0, kNB, false), 0);
      j0 += kNB;
      continue;
    }
    update(nf, j0, tiles(j0, kNB, true), 1);          // panel j -> panel j+1's columns
    panel(j0 + kNB);
    update(nf, j0, tiles(j0, 2 * kNB, false), 2);     // panels j, j+1 -> the rest
    j0 += 2 * kNB;
  }
  HIP_CHECK(hipGetLastError());
}

// One column-block step of apply_form: the fronts still active, the row
// tiles of the tallest, and how the finished columns are split over
// work-groups.  A step whose launch would hold fewer work-groups than the
// device has compute units (levels of few, large fronts: the top block, the
// upper 3D levels) splits its finished columns into ranges of whole panels,
// at most kInvSplitMax and at least four panels each.
constexpr int kInvSplitMax = 16;
// Apply-form variants: 0 column blocks on FMA, 1 column blocks on the
// matrix cores, 2 recursive doubling.
constexpr int INV_DOUBLING = 2;
static inline bool single_top(const std::vector<FrontDev>& fh) {
  return fh.size() == 1 && fh[0].s == fh[0].p;
}
// Apply-form variants open to the tuner (and to forcing) by type.
template <typename T> static inline int inv_variants() { return sizeof(T) == 8 ? 3 : 2; }
struct InvStep {
  int J = 0;
  unsigned na = 0;
  int64_t tiles = 0;
  int nsplit = 1, kchunk = 0;
};
static std::vector<InvStep> inv_steps(const std::vector<FrontDev>& fh, bool bounds, bool sorted) {
  std::vector<InvStep> out;
  int pmax = 0;
  for (const FrontDev& f : fh) pmax = std::max(pmax, f.p);
  for (int J = ((pmax - 1) / kNB) * kNB; J >= 0 && pmax > 0; J -= kNB) {
    InvStep s;
    s.J = J;
    int kblocks = 0;
    for (const auto& f : fh) {
      if (J >= f.p) continue;
      const int nb = bounds ? 1 : std::min(kNB, f.p - J);
      s.tiles = std::max<int64_t>(s.tiles, (f.s - J - nb + kIR - 1) / kIR);
      kblocks = std::max(kblocks, (f.p - J - std::min(kNB, f.p - J) + kNB - 1) / kNB);
    }
    s.na = active_fronts(fh, J, sorted);
    if (s.na == 0) continue;
    const int64_t wgs = int64_t(s.na) * s.tiles;
    if (s.tiles > 0 && wgs < 256 && kblocks >= 8) {
      const int want = int(std::min<int64_t>(kInvSplitMax, (512 + wgs - 1) / wgs));
      s.nsplit = std::max(1, std::min(want, kblocks / 4));
      const int per = (kblocks + s.nsplit - 1) / s.nsplit;
      s.kchunk = per * kNB;
      s.nsplit = (kblocks + per - 1) / per;
    }
    out.push_back(s);
  }
  return out;
}

// Buffers of apply_form: the column block of B in flight, s x kNB per front,
// each front's offset in it, and the partial residuals of split steps
// (nsplit x s x kNB per front, at the front's offset times nsplit).
template <typename T>
struct InvWork {
  T* tmp = nullptr;
  const int64_t* toff = nullptr;
  T* part = nullptr;
};
template <typename T>
static InvWork<T> apply_form_work(Arena& mem, const std::vector<FrontDev>& fh, hipStream_t st,
                                  bool bounds = false, bool sorted = true) {
  std::vector<int64_t> toff(fh.size());
  int64_t tot = 0;
  for (size_t i = 0; i < fh.size(); ++i) {
    toff[i] = tot;
    tot += int64_t(fh[i].s) * kNB;
  }
  int smax = 1;
  for (const InvStep& s : inv_steps(fh, bounds, sorted)) smax = std::max(smax, s.nsplit);
  InvWork<T> w;
  w.tmp = mem.get<T>(size_t(std::max<int64_t>(tot, 1)));
  w.toff = mem.upload(toff, st);
  if (smax > 1) w.part = mem.get<T>(size_t(tot) * size_t(smax));
  return w;
}

// With `work` prepared beforehand (apply_form_work on another stream),
// nothing is copied from the host here: a stream held behind an event can
// make a pageable host copy wait for that event.
template <typename T>
static void apply_form(Arena& mem, T* pool, const std::vector<FrontDev>& fh,
                       const FrontDev* fronts_d, hipStream_t st, bool bounds = false,
                       bool sorted = false, int variant = 1, const InvWork<T>* work = nullptr) {
  if (fh.empty()) return;
  if (variant == INV_DOUBLING && !bounds) {
    // recursive doubling for every front (exact pivot counts only)
    int pmax = 0;
    int64_t qpmax = 0;
    for (const FrontDev& f : fh) {
      pmax = std::max(pmax, f.p);
      qpmax = std::max<int64_t>(qpmax, int64_t(f.s - f.p) * f.p);
    }
    const unsigned nf = unsigned(fh.size());
    if (pmax == 0) return;
    hipLaunchKernelGGL(k_inv_mirror<T>, dim3(nf, unsigned((pmax + kNB - 1) / kNB)), dim3(kThreads),
                       0, st, pool, fronts_d);
    int64_t smax_tmp = 0;
    for (int64_t bs = kNB; bs < pmax; bs *= 2)
      smax_tmp = std::max<int64_t>(smax_tmp, ((pmax + 2 * bs - 1) / (2 * bs)) * bs * bs);
    if (smax_tmp > 0) {
      T* tmp = mem.get<T>(size_t(smax_tmp) * nf);
      for (int bs = kNB; bs < pmax; bs *= 2) {
        const int64_t pairs = (pmax + 2 * int64_t(bs) - 1) / (2 * int64_t(bs));
        const int64_t t1 = (bs + kTB - 1) / kTB;
        const int64_t stride = pairs * bs * bs;
        if (pairs * t1 * t1 > 65535) throw Error(HIFDE_EINVAL, "front too large for the doubling grid");
        for (int mode = 0; mode < 2; ++mode)
          hipLaunchKernelGGL(k_inv_double<T>, dim3(nf, unsigned(pairs * t1 * t1)), dim3(kThreads), 0,
                             st, pool, fronts_d, bs, tmp, stride, mode);
      }
    }
    if (qpmax > 0) {
      int qmax = 0;
      for (const FrontDev& f : fh) qmax = std::max(qmax, f.s - f.p);
      const int64_t tiles = int64_t((qmax + kTB - 1) / kTB) * ((pmax + kTB - 1) / kTB);
      if (tiles > 65535) throw Error(HIFDE_EINVAL, "front too large for the doubling grid");
      T* tq = mem.get<T>(size_t(qpmax) * nf);
      for (int mode = 0; mode < 2; ++mode)
        hipLaunchKernelGGL(k_inv_rows<T>, dim3(nf, unsigned(tiles)), dim3(kThreads), 0, st, pool,
                           fronts_d, tq, qpmax, mode);
    }
    HIP_CHECK(hipGetLastError());
    return;
  }
  if (variant == INV_DOUBLING) variant = 1;
  const InvWork<T> w = work ? *work : apply_form_work<T>(mem, fh, st, bounds, sorted);
  T* tmp = w.tmp;
  const int64_t* toff_d = w.toff;
  int smax = 0;
  for (const FrontDev& f : fh) smax = std::max(smax, f.s);
  const unsigned chunks = unsigned(std::max(1, (smax + kCommitRows - 1) / kCommitRows));
  for (const InvStep& s : inv_steps(fh, bounds, sorted)) {
    const int J = s.J;
    const unsigned na = s.na;
    const int64_t tiles = s.tiles;
    if (tiles > 0) {
      if (variant == 1 && s.nsplit > 1 && w.part) {
        const unsigned g = front_tile_grid(na, tiles * s.nsplit, "inversion grid");
        hipLaunchKernelGGL(k_inv_step_mfma<T>, dim3(g), dim3(kThreads), 0, st, pool, fronts_d, J,
                           tmp, toff_d, int(na), int(tiles * s.nsplit), s.nsplit, s.kchunk,
                           w.part);
        hipLaunchKernelGGL(k_inv_finish<T>, dim3(front_tile_grid(na, tiles, "inversion grid")),
                           dim3(kThreads), 0, st, pool, fronts_d, J, tmp, toff_d, int(na),
                           int(tiles), s.nsplit, static_cast<const T*>(w.part));
      } else if (variant == 1) {
        const unsigned g = front_tile_grid(na, tiles, "inversion grid");
        hipLaunchKernelGGL(k_inv_step_mfma<T>, dim3(g), dim3(kThreads), 0, st, pool, fronts_d, J,
                           tmp, toff_d, int(na), int(tiles), 1, 0, static_cast<T*>(nullptr));
      } else {
        const unsigned g = front_tile_grid(na, tiles, "inversion grid");
        hipLaunchKernelGGL(k_inv_step<T>, dim3(g), dim3(kThreads), 0, st, pool, fronts_d, J, tmp,
                           toff_d, int(na), int(tiles));
      }
    }
    // rows of the fronts still below J: chunks past a front's end return
    const unsigned ch = na < 64 ? chunks : 1u;
    hipLaunchKernelGGL(k_inv_commit<T>, dim3(na, ch), dim3(kThreads), 0, st, pool, fronts_d, J,
                       tmp, toff_d);
  }
  HIP_CHECK(hipGetLastError());
}

// Packed apply form and D^-1 of every front (the sweeps' copy).
// TP: the sweeps' type (float under the mixed precisions, double for the top
// block and in double precision).
template <typename T, typename TP = T>
static void pack_fronts(Arena& mem, const T* pool, const std::vector<FrontDev>& fh,
                        const FrontDev* fronts_d, const SweepSet& S, void** pk, void** pt,
                        void** dinv, hipStream_t st) {
  *pk = mem.get<TP>(size_t(std::max<int64_t>(S.pk_elems, 1)));
  *pt = mem.get<TP>(size_t(std::max<int64_t>(S.pt_elems, 1)));
  *dinv = mem.get<TP>(size_t(std::max<int64_t>(S.dv_elems, 1)));
  if (fh.empty()) return;
  int smax = 0;
  for (const FrontDev& f : fh) smax = std::max(smax, f.s);
  const unsigned rtmax = unsigned((smax + 15) / 16);
  if (rtmax > 65535) throw Error(HIFDE_EINVAL, "front too large for the packing grid");
  hipLaunchKernelGGL((k_pack<T, TP>), dim3(unsigned(fh.size()), std::max(1u, rtmax)), dim3(kThreads),
                     0, st, pool, fronts_d, S.packs, static_cast<TP*>(*pk), static_cast<TP*>(*pt),
                     static_cast<TP*>(*dinv));
  HIP_CHECK(hipGetLastError());
}

static PoolTable pools_for_level(const hifde_factor_s& F, int l_src) {
  PoolTable t{{nullptr, nullptr, nullptr}, {0, 0, 0}};
  if (l_src < 0) return t;
  t.p[POOL_CELLS] = F.cl[l_src].pool;
  t.esz[POOL_CELLS] = F.cl[l_src].esz;
  if (l_src < F.g.L) {
    t.p[POOL_BASE] = F.gl[l_src].base;
    t.p[POOL_FG] = F.gl[l_src].fg;
    t.esz[POOL_BASE] = t.esz[POOL_FG] = F.gl[l_src].esz;
  }
  return t;
}

// Elements of x a solve work-group can stage in LDS.

// Scratch for solve kernels whose x does not fit in LDS.

// LDS sizing of one solve launch: x capacity (elements) and bytes.

// ---------------------------------------------------------------------------
// Cells of level l: plan, assemble, factor.
// ---------------------------------------------------------------------------
// Autotuner: the variant of a launch family for a size bucket.  Without
// HIFDE_AUTOTUNE the tree's cached choice (or the default) is used; with it,
// an unseen bucket runs every variant once on a snapshot of the data it
// modifies (buf, bytes), timed with events, keeps the fastest for the tree,
// and restores the data for the real run.
enum { FAM_LDL = 1, FAM_CPQR = 2, FAM_INV = 3 };
constexpr int kCpqrWideFrom = 128;   // |c| from which the ID defaults to the wide form
constexpr int kSketchOversample = 16;   // rows of a sketch beyond |c|
constexpr int kAsmWideFrom = 512;    // front size from which extend-add goes wide
static uint64_t tune_key(int fam, int esz, int a, int b, int c) {
  auto bucket = [](int v) {
    int k = 0;
    while ((1 << k) < v) ++k;
    return uint64_t(k);
  };
  return (uint64_t(fam) << 56) | (uint64_t(esz) << 48) | (bucket(a) << 32) | (bucket(b) << 16) |
         bucket(c);
}

// HIFDE_TUNE_FORCE="ldl=<v>,cpqr=<v>" pins a family's variant (testing).
static int forced_variant(int fam) {
  const char* e = getenv("HIFDE_TUNE_FORCE");
  if (!e) return -1;
  const std::string s(e);
  const std::string name = fam == FAM_LDL ? "ldl=" : fam == FAM_CPQR ? "cpqr=" : "inv=";
  const size_t at = s.find(name);
  if (at == std::string::npos) return -1;
  return std::atoi(s.c_str() + at + name.size());
}

template <class Run>
static int tune_choice(hifde_factor_s& F, uint64_t key, int nvar, int dflt, void* buf,
                       size_t bytes, hipStream_t st, Run run, int ntime = -1) {
  // ntime: only variants below it are timed (the others can be forced)
  const int forced = forced_variant(int(key >> 56));
  if (forced >= 0 && forced < nvar) return forced;
  if (ntime < 0) ntime = nvar;
  hifde_tree_s* tree = F.tree;
  if (tree) {
    auto it = tree->tune.find(key);
    if (it != tree->tune.end()) return it->second;
  }
  if (!F.autotune || !tree || bytes == 0) return dflt;
  DevMem save;
  save.alloc(bytes);
  HIP_CHECK(hipMemcpyAsync(save.p, buf, bytes, hipMemcpyDeviceToDevice, st));
  hipEvent_t a = nullptr, b = nullptr;   // timing events, destroyed with F
  HIP_CHECK(hipEventCreate(&a));
  F.events.push_back(a);
  HIP_CHECK(hipEventCreate(&b));
  F.events.push_back(b);
  float best = 0.f;
  int bi = dflt;
  for (int v = 0; v < ntime; ++v) {
    // each variant twice, the faster run kept: a kernel's first launch in
    // the process also loads its code, which is no part of its cost
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      if (v > 0 || rep > 0)
        HIP_CHECK(hipMemcpyAsync(buf, save.p, bytes, hipMemcpyDeviceToDevice, st));
      HIP_CHECK(hipEventRecord(a, st));
      run(v);
      HIP_CHECK(hipEventRecord(b, st));
      HIP_CHECK(hipEventSynchronize(b));
      float t = 0.f;
      HIP_CHECK(hipEventElapsedTime(&t, a, b));
      ms = rep == 0 ? t : std::min(ms, t);
    }
    if (getenv("HIFDE_TIMING"))
      fprintf(stderr, "[hifde] tune family %d key %016llx variant %d: %.3f ms\n", int(key >> 56),
              static_cast<unsigned long long>(key), v, ms);
    if (v == 0 || ms < best) {
      best = ms;
      bi = v;
    }
  }
  HIP_CHECK(hipMemcpyAsync(buf, save.p, bytes, hipMemcpyDeviceToDevice, st));
  HIP_CHECK(hipStreamSynchronize(st));
  tree->tune[key] = bi;
  F.tuned += 1;
  return bi;
}

// Fronts sorted by pivot count, descending (bucketed launches).
static std::vector<FrontDev> sorted_by_p(const std::vector<FrontDev>& fh) {
  std::vector<FrontDev> out(fh);
  std::stable_sort(out.begin(), out.end(),
                   [](const FrontDev& x, const FrontDev& y) { return x.p > y.p; });
  return out;
}

// T: the type the cells are eliminated in; TP: the type of their packed
// apply form (the sweeps' type).
template <typename T, typename TP>
static void cells_level(hifde_factor_s& F, hifde_tree_s* tree, int l, hipStream_t st) {
  Planner& P = *F.planner;
  CellLevel& D = F.cl[l];
  D.esz = int(sizeof(T));
  PhaseTimer tm;
  if (l == 0 && tree->c0) {
    F.join_skel();
    F.flush_side(st);
    D.st = tree->c0;
  } else {
    if (l > 0) P.plan_cells(l);
    tm.mark("  plan cells", l);
    F.join_skel();   // the previous level's skeleton fronts
    F.flush_side(st);
    D.st = make_cell_static(F, *P.level(l).plan, l == 0);
    tm.mark("  cell descriptors", l);
    if (l == 0) {
      tree->c0 = D.st;
      tree->c0_esz = sizeof(T);   // (the type its cells were first eliminated in)
    }
  }
  if (F.plan_only) return;
  CellStatic& S = *D.st;
  upload_cell_static(S, l == 0 ? S.mem : F.mem, st);
  // fronts of the narrow assembly clear their own lower triangles (the
  // only part later steps read before writing); the wide form needs the
  // pool cleared first (level 0 of a known tree: allocated up front)
  const bool wide_asm = S.smax >= kAsmWideFrom;
  if (!D.pool) {
    D.pool = F.mem.get<T>(size_t(S.elems));
    if (wide_asm) HIP_CHECK(hipMemsetAsync(D.pool, 0, size_t(S.elems) * sizeof(T), st));
  }
  D.info = F.mem.get<int>(std::max(1, S.ncell));
  HIP_CHECK(hipMemsetAsync(D.info, 0, sizeof(int) * std::max(1, S.ncell), st));
  PoolTable pt = pools_for_level(F, l - 1);
  if (S.ncell > 0) {
    if (S.smax >= kAsmWideFrom) {
      // large fronts: one launch per source round, columns over work-groups
      int rounds = 0, dmax = 0;
      int64_t tmax = 0;
      for (const FrontDev& f : S.fh) {
        rounds = std::max(rounds, f.src_end - f.src_begin);
        tmax = std::max<int64_t>(tmax, f.trip_end - f.trip_begin);
      }
      for (const SrcDev& d : S.srcs_h) dmax = std::max(dmax, d.dim);
      const AsmChunks ch = asm_chunks(S.ncell, dmax);
      for (int r = 0; r < rounds; ++r)
        hipLaunchKernelGGL((k_assemble_round<T>),
                           dim3(S.ncell, (dmax + ch.cols - 1) / ch.cols,
                                (dmax + ch.rows - 1) / ch.rows),
                           dim3(kThreads), 0, st, static_cast<T*>(D.pool), S.fronts, S.srcs, S.maps,
                           r, pt, ch.cols, ch.rows);
      if (tmax > 0)
        hipLaunchKernelGGL(k_assemble_trips<T>, dim3(S.ncell, unsigned((tmax + 4095) / 4096)),
                           dim3(kThreads), 0, st, static_cast<T*>(D.pool), S.fronts, S.trips,
                           F.diag.as<double>(), F.offd.as<double>(), F.g.N);
    } else {
      hipLaunchKernelGGL((k_assemble<T>), dim3(S.ncell), dim3(kThreads), 0, st,
                         static_cast<T*>(D.pool), S.fronts, S.srcs, S.maps, S.trips,
                         F.diag.as<double>(), F.offd.as<double>(), F.g.N, pt, 1);
    }
  }
  HIP_CHECK(hipGetLastError());
  // elimination and apply form in buckets of pivot count (sorted fronts)
  std::vector<FrontDev> fs = sorted_by_p(S.fh);
  const FrontDev* fs_d = F.mem.upload(fs, st);
  // the apply form's buffers (uploaded here, before the elimination is
  // queued: see apply_form)
  const InvWork<T> iw = apply_form_work<T>(F.mem, fs, st);
  int* ldl_counter = F.mem.get<int>(1);
  const int var = tune_choice(
      F, tune_key(FAM_LDL, int(sizeof(T)), S.pmax, S.smax, S.ncell), LDL_VARIANTS, LDL_MFMA, D.pool,
      size_t(S.elems) * sizeof(T), st, [&](int v) {
        batched_ldl<T>(static_cast<T*>(D.pool), fs, fs_d, D.info, F.definite, st, false, true, v,
                       ldl_counter, S.env, S.pband);
      }, ldl_timed(S.ncell));
  batched_ldl<T>(static_cast<T*>(D.pool), fs, fs_d, D.info, F.definite, st, false, true, var,
                 ldl_counter, S.env, S.pband);
  // The apply form and its packed copy are read by the sweeps only: they run
  // on the side stream after this level's IDs, beside the host's skeleton
  // bookkeeping and the next level's planning.  They touch the first p
  // columns of each front; the groups and later levels read the update
  // blocks.
  F.side_work = [&F, &D, &S, fs = std::move(fs), fs_d, iw](hipStream_t ss) {
    // the top block (one front, no trailing block) defaults to the doubling
    // form from 256 pivots on; float fronts keep the column blocks (the
    // doubling's products of inverted blocks round less favourably there,
    // which shows on indefinite fronts)
    const int ivar = tune_choice(
        F, tune_key(FAM_INV, int(sizeof(T)), S.pmax, S.smax, S.ncell), inv_variants<T>(),
        single_top(fs) && fs[0].p >= 256 ? INV_DOUBLING : 1, D.pool,
        size_t(S.elems) * sizeof(T), ss, [&](int v) {
          apply_form<T>(F.mem, static_cast<T*>(D.pool), fs, fs_d, ss, false, true, v, &iw);
        });
    apply_form<T>(F.mem, static_cast<T*>(D.pool), fs, fs_d, ss, false, true, ivar, &iw);
    pack_fronts<T, TP>(F.mem, static_cast<const T*>(D.pool), S.fh, S.fronts, S.sw, &D.pk, &D.pt,
                       &D.dinv, ss);
  };
}

// The input flags of k_stencil (read once, at the first synchronization).
static void check_input(hifde_factor_s& F, hipStream_t st) {
  if (F.input_checked || !F.bad_d) return;
  int* hp = static_cast<int*>(F.host_stage(sizeof(int)));
  HIP_CHECK(hipMemcpyAsync(hp, F.bad_d, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  const int h = *hp;
  F.input_checked = true;
  if (h & 1)
    throw Error(HIFDE_EINVAL, "a must be finite, positive on interior links, >= 0 on boundary links");
  if (h & 2) throw Error(HIFDE_EINVAL, "b must be finite");
}

static void report_info(const std::vector<int>& h, const char* what, int l, bool definite) {
  for (size_t i = 0; i < h.size(); ++i)
    if (h[i] != 0) {
      char buf[200];
      snprintf(buf, sizeof buf, "%s pivot in %s %zu of level %d (panel at %d)",
               definite ? "non-positive" : "zero or non-finite", what, i, l, h[i] - 1);
      throw Error(HIFDE_ENOTSPD, buf);
    }
}

// Pivot flags of the level-l cells and of the level l-1/2 skeleton fronts,
// queued for the host beside the level's ranks: a block that is not positive
// definite stops the factorization at the first synchronization after it
// rather than after every later level.
struct LevelPivots {
  std::vector<int> cells, groups;
  const int* cinfo = nullptr;
  const int* ginfo = nullptr;
  // the flag counts of level l (sizes the vectors); ints to stage
  size_t count(const hifde_factor_s& F, int l) {
    const CellLevel& C = F.cl[l];
    cinfo = ginfo = nullptr;
    cells.clear();
    groups.clear();
    if (C.info && C.st) {
      cells.resize(C.st->fh.size());
      cinfo = C.info;
    }
    if (l > 0 && F.gl[l - 1].info) {
      const GroupLevel& G = F.gl[l - 1];
      groups.resize(F.presize ? size_t(G.ngroup) : size_t(G.nskel));
      ginfo = G.info;
    }
    return cells.size() + groups.size();
  }
  // copies into the pinned `stage` (count() ints)
  void queue(int* stage, hipStream_t st) const {
    if (!cells.empty())
      HIP_CHECK(hipMemcpyAsync(stage, cinfo, cells.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    if (!groups.empty())
      HIP_CHECK(hipMemcpyAsync(stage + cells.size(), ginfo, groups.size() * sizeof(int),
                               hipMemcpyDeviceToHost, st));
  }
  // after the stream has synchronized
  void collect(const int* stage) {
    std::copy(stage, stage + cells.size(), cells.begin());
    std::copy(stage + cells.size(), stage + cells.size() + groups.size(), groups.begin());
  }
  void check(int l, bool definite) const {   // after the stream has synchronized
    report_info(cells, "cell", l, definite);
    report_info(groups, "group", l - 1, definite);
  }
};

// ---------------------------------------------------------------------------
// Groups of level l+1/2: plan, base blocks, ID, skeleton fronts.
// ---------------------------------------------------------------------------
// Device features of the groups of level l+1/2 (kRankF floats per group,
// into feat) from the planned groups' [c^N; c] lists and the stencil.
static void group_features(hifde_factor_s& F, int l, float* feat, hipStream_t st) {
  const auto& groups = F.planner->level(l).groups();
  if (groups.empty()) return;
  std::vector<int32_t> lists, nn, nc;
  std::vector<int64_t> offs;
  for (const Group& g : groups) {
    offs.push_back(int64_t(lists.size()));
    lists.insert(lists.end(), g.cN.begin(), g.cN.end());
    lists.insert(lists.end(), g.c.begin(), g.c.end());
    nn.push_back(int32_t(g.cN.size()));
    nc.push_back(int32_t(g.c.size()));
  }
  const int32_t* ld = F.mem.upload(lists, st);
  const int64_t* od = F.mem.upload(offs, st);
  const int32_t* nnd = F.mem.upload(nn, st);
  const int32_t* ncd = F.mem.upload(nc, st);
  hipLaunchKernelGGL(k_rank_features, dim3(unsigned(groups.size())), dim3(kThreads), 0, st, ld, od,
                     nnd, ncd, F.offd.as<double>(), F.g.N, F.g.n, F.g.dim, F.eps, l, feat);
  HIP_CHECK(hipGetLastError());
}

// Rank-model inference for the groups of level l+1/2 on the auxiliary
// stream (it overlaps the level's eliminations): features, network,
// ranks, an asynchronous copy to page-locked memory and an event.
static void predict_ranks(hifde_factor_s& F, GroupLevel& G, int l) {
  const int ng = G.ngroup;
  if (ng == 0) return;
  if (!F.aux) {
    F.aux = StreamCache::get().take();
  }
  HIP_CHECK(hipStreamWaitEvent(F.aux, F.offd_ev, 0));
  float* feat = F.mem.get<float>(size_t(ng) * kRankF);
  float* y = F.mem.get<float>(ng);
  std::vector<int32_t> nc(ng);
  for (int g = 0; g < ng; ++g) nc[g] = G.gh[g].nc;
  const int32_t* ncd = F.mem.upload(nc, F.aux);
  G.khat_d = F.mem.get<int32_t>(ng);
  group_features(F, l, feat, F.aux);
  hipLaunchKernelGGL(k_mlp_forward, dim3(nblk(ng)), dim3(kThreads), 0, F.aux, F.model, int64_t(ng),
                     feat, y, static_cast<float*>(nullptr), static_cast<float*>(nullptr));
  hipLaunchKernelGGL(k_rank_from_output, dim3(nblk(ng)), dim3(kThreads), 0, F.aux, ng, y, ncd,
                     G.khat_d);
  G.khat_h = std::make_shared<PinnedMem>();
  G.khat_h->ensure(size_t(ng) * 4);
  HIP_CHECK(hipMemcpyAsync(G.khat_h->p, G.khat_d, size_t(ng) * 4, hipMemcpyDeviceToHost, F.aux));
  G.pred_ev = F.new_event();
  HIP_CHECK(hipEventRecord(G.pred_ev, F.aux));
  HIP_CHECK(hipGetLastError());
}

// Skeleton fronts: one work-group per group, or for large groups two
// launches (B_sr and E columns, then B_rr columns) over column chunks.
template <typename T>
static void launch_group_front(GroupLevel& G, int nblocks, int ncmax, const int32_t* gsel,
                               const int32_t* kdev, hipStream_t st) {
  if (ncmax < kCpqrWideFrom) {
    hipLaunchKernelGGL(k_group_front<T>, dim3(nblocks), dim3(kThreads), 0, st,
                       static_cast<T*>(G.fg), static_cast<const T*>(G.gw),
                       static_cast<const T*>(G.base), static_cast<const T*>(G.tpool), G.groups,
                       G.perm, G.perm_stride, gsel, kdev, -1);
  } else {
    // large groups on the matrix cores: output tiles of 64 x 64 (bounds from
    // |c|, since the ranks may still be on the device)
    const int64_t tb = (ncmax + kTB - 1) / kTB;
    const unsigned t0 = unsigned(std::max<int64_t>(1, tb * tb));
    const unsigned t1 = unsigned(std::max<int64_t>(1, tb * (tb + 1) / 2));
    if (t0 > 65535) throw Error(HIFDE_EINVAL, "group too large for the skeleton-front grid");
    hipLaunchKernelGGL(k_group_front_mfma<T>, dim3(nblocks, t0), dim3(kThreads), 0, st,
                       static_cast<T*>(G.fg), static_cast<const T*>(G.gw),
                       static_cast<const T*>(G.base), static_cast<const T*>(G.tpool), G.groups,
                       G.perm, G.perm_stride, gsel, kdev, 0);
    hipLaunchKernelGGL(k_group_front_mfma<T>, dim3(nblocks, t1), dim3(kThreads), 0, st,
                       static_cast<T*>(G.fg), static_cast<const T*>(G.gw),
                       static_cast<const T*>(G.base), static_cast<const T*>(G.tpool), G.groups,
                       G.perm, G.perm_stride, gsel, kdev, 1);
  }
  HIP_CHECK(hipGetLastError());
}

// The skeleton fronts of level l (Lemma 2.4) once its ranks are known: the
// groups' lists, the fronts' assembly, elimination and apply form, and
// their sweep descriptors.  Run on a helper thread beside the planning of
// level l+1 (it uses the arena and the stream; the main thread waits for
// it before it does).
template <typename T>
static void skeleton_fronts(hifde_factor_s& F, GroupLevel& G, const Level& lev,
                           const std::vector<int32_t>& kh, int l, hipStream_t st) {
  PhaseTimer tm;
  int64_t fg_off = 0;
  int rmax = 0;
  {
    size_t nidx = 0, nsk = 0;
    for (int gi = 0; gi < G.ngroup; ++gi)
      if (kh[gi] < G.gh[gi].nc) {
        nidx += size_t(G.gh[gi].nc);
        nsk += 1;
      }
    G.idx_h.reserve(nidx);
    G.ff.reserve(nsk);
    G.gsel_h.reserve(nsk);
  }
  for (int gi = 0; gi < G.ngroup; ++gi) {
    GroupDev& d = G.gh[gi];
    const int k = kh[gi];
    d.k = k;
    d.skel = (k < d.nc) ? 1 : 0;
    if (!d.skel) continue;
    d.fg_off = fg_off;
    G.tel += double(k) * (d.nc - k);
    G.rrows += d.nc - k;
    G.krows += k;
    rmax = std::max(rmax, d.nc - k);
    FrontDev f{};
    f.off = d.fg_off;
    f.s = d.nc;
    f.p = d.nc - k;
    f.idx = int64_t(G.idx_h.size());
    G.ff.push_back(f);
    fg_off += int64_t(d.nc) * d.nc;
    d.idx = int64_t(G.idx_h.size());
    const GroupRes& R = lev.res[gi];
    G.idx_h.insert(G.idx_h.end(), R.rd.begin(), R.rd.end());
    G.idx_h.insert(G.idx_h.end(), R.sk.begin(), R.sk.end());
    G.gsel_h.push_back(gi);
    G.ncskel = std::max(G.ncskel, int(d.nc));
  }
  tm.mark("  skeleton lists", l);
  G.nskel = int(G.gsel_h.size());
  G.groups = F.mem.upload(G.gh, st);
  if (G.nskel == 0) return;
  G.idx = F.mem.upload(G.idx_h, st);
  G.gsel = F.mem.upload(G.gsel_h, st);
  G.fg = F.mem.get<T>(size_t(fg_off));
  HIP_CHECK(hipMemsetAsync(G.fg, 0, size_t(fg_off) * sizeof(T), st));
  G.fgfronts = F.mem.upload(G.ff, st);
  G.info = F.mem.get<int>(G.ff.size());
  HIP_CHECK(hipMemsetAsync(G.info, 0, sizeof(int) * G.ff.size(), st));
  launch_group_front<T>(G, G.nskel, G.ncskel, G.gsel, static_cast<const int32_t*>(nullptr), st);
  {
    const std::vector<FrontDev> fs = sorted_by_p(G.ff);
    const FrontDev* fs_d = F.mem.upload(fs, st);
    int* ldl_counter = F.mem.get<int>(1);
    int pmx = 0, smx = 0;
    for (const FrontDev& f : fs) {
      pmx = std::max(pmx, f.p);
      smx = std::max(smx, f.s);
    }
    const int var = tune_choice(
        F, tune_key(FAM_LDL, int(sizeof(T)), pmx, smx, G.nskel), LDL_VARIANTS, LDL_MFMA, G.fg,
        size_t(fg_off) * sizeof(T), st, [&](int v) {
          batched_ldl<T>(static_cast<T*>(G.fg), fs, fs_d, G.info, F.definite, st, false, true, v,
                         ldl_counter);
        }, ldl_timed(G.nskel));
    batched_ldl<T>(static_cast<T*>(G.fg), fs, fs_d, G.info, F.definite, st, false, true, var,
                   ldl_counter);
    const int ivar = tune_choice(
        F, tune_key(FAM_INV, int(sizeof(T)), pmx, smx, G.nskel), inv_variants<T>(), 1, G.fg,
        size_t(fg_off) * sizeof(T), st,
        [&](int v) { apply_form<T>(F.mem, static_cast<T*>(G.fg), fs, fs_d, st, false, true, v); });
    apply_form<T>(F.mem, static_cast<T*>(G.fg), fs, fs_d, st, false, true, ivar);
  }
  F.skel_panels += (rmax + kNB - 1) / kNB;
  build_sweep(G.sw, G.ff, false);
  for (size_t i = 0; i < G.sw.ph.size(); ++i) G.sw.ph[i].t_off = G.gh[G.gsel_h[i]].t_off;
  upload_sweep(G.sw, F.mem, st);
  pack_fronts<T>(F.mem, static_cast<const T*>(G.fg), G.ff, G.fgfronts, G.sw, &G.pk, &G.pt,
                 &G.dinv, st);
  tm.mark("  skeleton fronts", l);
}

template <typename T>
static void groups_level(hifde_factor_s& F, hifde_tree_s* tree, int l, hipStream_t st) {
  Planner& P = *F.planner;
  const bool skel = F.eps > 0.0 && l >= F.g.skip;
  GroupLevel& G = F.gl[l];
  G.esz = int(sizeof(T));
  PhaseTimer tm;
  P.plan_groups(l);
  tm.mark("  plan groups", l);
  if (l == 0 && tree->g0 && (tree->g0->gw_elems > 0) == skel) {
    G.st = tree->g0;
  } else {
    G.st = make_group_static(F, *P.level(l).plan, skel);
    if (l == 0) tree->g0 = G.st;
  }
  tm.mark("  group descriptors", l);
  GroupStatic& S = *G.st;
  G.gh = S.gh;
  G.ngroup = int(G.gh.size());
  const Level& lev = P.level(l);
  if (F.plan_only) return;
  const bool pre = skel && F.presize != 0 && G.ngroup > 0;
  if (pre && F.presize == 1) predict_ranks(F, G, l);
  upload_group_static(S, l == 0 ? S.mem : F.mem, st);
  G.base = F.mem.get<T>(size_t(S.base_elems));
  HIP_CHECK(hipMemsetAsync(G.base, 0, size_t(S.base_elems) * sizeof(T), st));
  PoolTable pt_prev = pools_for_level(F, l - 1);
  if (G.ngroup > 0) {
    hipLaunchKernelGGL((k_assemble<T>), dim3(G.ngroup), dim3(kThreads), 0, st,
                       static_cast<T*>(G.base), S.bfronts, S.bsrcs, S.maps, S.btrips,
                       F.diag.as<double>(), F.offd.as<double>(), F.g.N, pt_prev, 0);
    HIP_CHECK(hipGetLastError());
  }
  tm.mark("  group bases", l);
  if (!skel || G.ngroup == 0) {
    F.flush_side(st);
    for (int gi = 0; gi < G.ngroup; ++gi) P.set_skeleton(l, gi, G.gh[gi].nc, nullptr);
    P.finish_groups(l);
    G.nskel = 0;
    return;
  }
  G.gw = F.mem.get<T>(size_t(S.gw_elems));
  HIP_CHECK(hipMemsetAsync(G.gw, 0, size_t(S.gw_elems) * sizeof(T), st));
  G.tpool = F.mem.get<T>(size_t(S.t_elems));
  HIP_CHECK(hipMemsetAsync(G.tpool, 0, size_t(S.t_elems) * sizeof(T), st));
  // with pre-launch every group owns a skeleton-front slot from the start
  int64_t fg_all = 0;
  if (pre)
    for (GroupDev& d : G.gh) {
      d.fg_off = fg_all;
      fg_all += int64_t(d.nc) * d.nc;
    }
  G.groups = F.mem.upload(G.gh, st);
  PoolTable pt_cur{{F.cl[l].pool, nullptr, nullptr}, {F.cl[l].esz, 0, 0}};
  const int ncmax = S.ncmax;
  if (ncmax >= kCpqrWideFrom) {
    // large groups: source rounds, base block, loose links over column chunks
    int rounds = 0, dmax = 0;
    int64_t tmax = 0;
    for (const GroupDev& d : G.gh) {
      rounds = std::max(rounds, d.src_end - d.src_begin);
      tmax = std::max<int64_t>(tmax, d.trip_end - d.trip_begin);
    }
    for (const SrcDev& d : S.gsrcs_h) dmax = std::max(dmax, d.dim);
    const unsigned ng = unsigned(G.ngroup);
    const AsmChunks ch = asm_chunks(ng, dmax);
    for (int r = 0; r < rounds; ++r)
      hipLaunchKernelGGL(k_gather_round<T>,
                         dim3(ng, (dmax + ch.cols - 1) / ch.cols, (dmax + ch.rows - 1) / ch.rows),
                         dim3(kThreads), 0, st, static_cast<T*>(G.gw), G.groups, S.gsrcs, S.maps, r,
                         pt_cur, ch.cols, ch.rows);
    hipLaunchKernelGGL(k_gather_base<T>, dim3(ng, (ncmax + kAsmCols - 1) / kAsmCols),
                       dim3(kThreads), 0, st, static_cast<T*>(G.gw),
                       static_cast<const T*>(G.base), G.groups);
    if (tmax > 0)
      hipLaunchKernelGGL(k_gather_trips<T>, dim3(ng, unsigned((tmax + 4095) / 4096)),
                         dim3(kThreads), 0, st, static_cast<T*>(G.gw), G.groups, S.gtrips,
                         F.diag.as<double>(), F.offd.as<double>(), F.g.N);
  } else {
    hipLaunchKernelGGL(k_group_gather<T>, dim3(G.ngroup), dim3(kThreads), 0, st,
                       static_cast<T*>(G.gw), static_cast<const T*>(G.base), G.groups, S.gsrcs,
                       S.maps, S.gtrips, F.diag.as<double>(), F.offd.as<double>(), F.g.N, pt_cur);
  }
  HIP_CHECK(hipGetLastError());
  tm.mark("  gather", l);
  // Randomized compression (Section 4.3): a group with |c^N| > |c| + 16 runs
  // its ID on the sketch Y = Phi M of r = |c| + 16 rows; the others on a copy
  // of M.  The IDs then read a workspace of their own, described by idh.
  T* idw = static_cast<T*>(G.gw);
  const GroupDev* idg = G.groups;
  const std::vector<GroupDev>* idh = &G.gh;
  size_t id_elems = size_t(S.gw_elems);
  std::vector<GroupDev> sgh;
  if (F.sketch) {
    const auto& pg = P.level(l).groups();
    std::vector<SketchDev> sk(G.ngroup);
    sgh = G.gh;
    int64_t yoff = 0, poff = 0, tiles = 1;
    for (int g = 0; g < G.ngroup; ++g) {
      const GroupDev& d = G.gh[g];
      SketchDev& k = sk[g];
      k.m_off = d.gw_off;
      k.nn = d.nn;
      k.nc = d.nc;
      k.r = std::min<int>(d.nn, d.nc + kSketchOversample);
      k.gid = uint32_t(pg[g].gid);
      k.y_off = yoff;
      if (k.r < k.nn) {
        k.phi_off = poff;
        poff += int64_t(k.r) * k.nn;
      } else {
        k.phi_off = -1;
      }
      yoff += (int64_t(k.r) + k.nc) * k.nc;
      tiles = std::max<int64_t>(tiles, int64_t((k.r + 63) / 64) * ((k.nc + 63) / 64));
      sgh[g].gw_off = k.y_off;
      sgh[g].nn = k.r;
    }
    T* phi = F.mem.get<T>(size_t(std::max<int64_t>(poff, 1)));
    idw = F.mem.get<T>(size_t(std::max<int64_t>(yoff, 1)));
    id_elems = size_t(yoff);
    const SketchDev* sk_d = F.mem.upload(sk, st);
    idg = F.mem.upload(sgh, st);
    idh = &sgh;
    if (poff > 0)
      hipLaunchKernelGGL(k_sketch_gen<T>, dim3(G.ngroup, 64), dim3(kThreads), 0, st, phi, sk_d,
                         l);
    hipLaunchKernelGGL(k_sketch_mfma<T>, dim3(G.ngroup, unsigned(tiles)), dim3(kThreads), 0, st,
                       static_cast<const T*>(G.gw), static_cast<const T*>(phi), idw, sk_d);
    HIP_CHECK(hipGetLastError());
    tm.mark("  sketch", l);
  }
  G.perm_stride = ncmax;
  G.kout = F.mem.get<int32_t>(G.ngroup);
  G.perm = F.mem.get<int32_t>(size_t(G.ngroup) * ncmax);
  const size_t smem = size_t(ncmax) * (sizeof(T) + 2 * sizeof(int));
  if (smem > 64 * 1024)
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cpqr<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(smem)));
  if (smem > 64 * 1024) {
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cpqr_queue<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(smem)));
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cpqr_1k<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(smem)));
  }
  const double tau = sizeof(T) == 8 ? 1e-10 : 1e-5;
  {
    // queue order: largest work (|c^N| |c|^2) first
    std::vector<int32_t> order(G.ngroup);
    for (int g = 0; g < G.ngroup; ++g) order[g] = g;
    int nnmax = 0;
    for (const GroupDev& d : *idh) nnmax = std::max(nnmax, int(d.nn));
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      const GroupDev &a = (*idh)[x], &b = (*idh)[y];
      return double(a.nn + a.nc) * a.nc * a.nc > double(b.nn + b.nc) * b.nc * b.nc;
    });
    const int32_t* order_d = F.mem.upload(order, st);
    int* counter = F.mem.get<int>(1);
    int dev = 0, ncu = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned qgrid = unsigned(std::min(G.ngroup, std::max(1, ncu) * 4));
    // wide form: every group of the launch, all steps in lock-step
    int maxsteps = 0;
    std::vector<int64_t> noff(G.ngroup);
    int64_t ntot = 0;
    for (int g = 0; g < G.ngroup; ++g) {
      noff[g] = ntot;
      ntot += (*idh)[g].nc;
      maxsteps = std::max(maxsteps, std::min<int>((*idh)[g].nn, (*idh)[g].nc));
    }
    auto run_wide = [&] {
      std::vector<int32_t> list(G.ngroup);
      for (int g = 0; g < G.ngroup; ++g) list[g] = g;
      const int32_t* list_d = F.mem.upload(list, st);
      const int64_t* noff_d = F.mem.upload(noff, st);
      T* norms = F.mem.get<T>(size_t(std::max<int64_t>(ntot, 1)));
      int32_t* permw = F.mem.get<int32_t>(size_t(std::max<int64_t>(ntot, 1)));
      CpqrWide<T>* stw = F.mem.get<CpqrWide<T>>(G.ngroup);
      int* live_d = F.mem.get<int>(1);
      const unsigned ng = unsigned(G.ngroup);
      const unsigned chunks = unsigned((ncmax + kCpqrChunk - 1) / kCpqrChunk);
      // LDS of the update: the reflector's rows when they fit the register path
      const size_t upd_lds = size_t(std::min(nnmax, 64 * kCpqrRegRows)) * sizeof(T);
      if (upd_lds > 64 * 1024)
        HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cpqr_w_update<T>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(upd_lds)));
      hipLaunchKernelGGL(k_cpqr_w_init<T>, dim3(ng, chunks), dim3(kThreads), 0, st,
                         idw, idg, list_d, norms, noff_d, permw, stw);
      // the host waits inside the step loop (the rank checks below): the
      // side stream's work is released now so that it runs beside the steps
      // (few work-groups each) instead of after them
      F.flush_side(st);
      for (int j = 0; j < maxsteps; ++j) {
        hipLaunchKernelGGL(k_cpqr_w_pivot<T>, dim3(ng), dim3(kThreads), 0, st,
                           idw, idg, list_d, norms, noff_d, permw, stw, j,
                           F.eps, tau);
        const unsigned uch = unsigned(std::max(1, (ncmax - j - 1 + kCpqrChunk - 1) / kCpqrChunk));
        hipLaunchKernelGGL(k_cpqr_w_update<T>, dim3(ng, uch), dim3(kThreads), upd_lds, st,
                           idw, idg, list_d, norms, noff_d, stw, j);
        if ((j & 31) == 31) {   // stop once every group has its rank
          int* live = static_cast<int*>(F.host_stage(sizeof(int)));
          hipLaunchKernelGGL(k_cpqr_w_live<T>, dim3(1), dim3(kThreads), 0, st, stw, G.ngroup,
                             live_d);
          HIP_CHECK(hipMemcpyAsync(live, live_d, sizeof(int), hipMemcpyDeviceToHost, st));
          HIP_CHECK(hipStreamSynchronize(st));
          if (*live == 0) break;
        }
      }
      // columns per work-group of the triangular solve: as many as the LDS
      // holds for the largest possible rank
      const int kmax = std::max(1, std::min(nnmax, ncmax));
      int cw = 64;
      while (cw > 1 && size_t(cw + 3) * kmax * sizeof(T) > 64 * 1024) cw /= 2;
      const size_t ts_lds = size_t(cw + 3) * kmax * sizeof(T);
      if (ts_lds > 160 * 1024) throw Error(HIFDE_EINVAL, "group too large for the ID's solve");
      if (ts_lds > 64 * 1024)
        HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cpqr_w_tsolve<T>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(ts_lds)));
      hipLaunchKernelGGL(k_cpqr_w_tsolve<T>, dim3(ng, unsigned((ncmax + cw - 1) / cw)),
                         dim3(kThreads), ts_lds, st, idw, idg, list_d, stw, cw);
      hipLaunchKernelGGL(k_cpqr_w_finish<T>, dim3(ng), dim3(kThreads), size_t(ncmax) * sizeof(int),
                         st, idw, static_cast<T*>(G.tpool), idg, list_d,
                         noff_d, permw, stw, G.kout, G.perm, G.perm_stride);
      HIP_CHECK(hipGetLastError());
    };
    auto run = [&](int v) {
      if (v == 2) {
        run_wide();
        return;
      }
      if (v == 3) {
        hipLaunchKernelGGL(k_cpqr_1k<T>, dim3(G.ngroup), dim3(1024), smem, st,
                           idw, static_cast<T*>(G.tpool), idg, F.eps, tau,
                           G.kout, G.perm, G.perm_stride);
        HIP_CHECK(hipGetLastError());
        return;
      }
      if (v == 1) {
        HIP_CHECK(hipMemsetAsync(counter, 0, sizeof(int), st));
        hipLaunchKernelGGL(k_cpqr_queue<T>, dim3(qgrid), dim3(kThreads), smem, st,
                           idw, static_cast<T*>(G.tpool), idg, F.eps, tau,
                           G.kout, G.perm, G.perm_stride, order_d, G.ngroup, counter);
      } else {
        hipLaunchKernelGGL(k_cpqr<T>, dim3(G.ngroup), dim3(kThreads), smem, st,
                           idw, static_cast<T*>(G.tpool), idg, F.eps, tau,
                           G.kout, G.perm, G.perm_stride);
      }
      HIP_CHECK(hipGetLastError());
    };
    // default: the wide form once groups are too large for one work-group
    const int dflt = ncmax >= kCpqrWideFrom ? 2 : G.ngroup < 256 ? 3 : 0;
    const int var = tune_choice(F, tune_key(FAM_CPQR, int(sizeof(T)), ncmax, nnmax, G.ngroup), 4,
                                dflt, idw, id_elems * sizeof(T), st, run);
    run(var);
  }

  // Pre-launch: the skeleton fronts of every group are formed, eliminated,
  // turned into the apply form and packed before the ranks reach the host.
  // The pivot count of each front comes from the IDs on the device; the
  // host bounds the panel sweeps by the predicted (or worst-case) ranks.
  std::vector<FrontDev> fall;
  SweepSet sall;
  std::vector<int32_t> khat;
  int pbound = 0;
  auto launch_fronts = [&](int bound) {
    for (FrontDev& f : fall) f.p = std::min(f.s, bound);
    G.fgfronts = F.mem.upload(fall, st);
    upload_sweep(sall, F.mem, st);
    hipLaunchKernelGGL(k_fix_fronts, dim3(nblk(G.ngroup)), dim3(kThreads), 0, st, G.ngroup, G.kout,
                       G.fgfronts, sall.packs);
    HIP_CHECK(hipMemsetAsync(G.fg, 0, size_t(fg_all) * sizeof(T), st));
    HIP_CHECK(hipMemsetAsync(G.info, 0, sizeof(int) * G.ngroup, st));
    launch_group_front<T>(G, G.ngroup, ncmax, static_cast<const int32_t*>(nullptr), G.kout, st);
    batched_ldl<T>(static_cast<T*>(G.fg), fall, G.fgfronts, G.info, F.definite, st, true);
    apply_form<T>(F.mem, static_cast<T*>(G.fg), fall, G.fgfronts, st, true);
    F.skel_panels += (bound + kNB - 1) / kNB;
    pack_fronts<T>(F.mem, static_cast<const T*>(G.fg), fall, G.fgfronts, sall, &G.pk, &G.pt,
                   &G.dinv, st);
  };
  if (pre) {
    khat.assign(G.ngroup, 0);
    if (F.presize == 1) {
      HIP_CHECK(hipEventSynchronize(G.pred_ev));
      std::copy(G.khat_h->as<int32_t>(), G.khat_h->as<int32_t>() + G.ngroup, khat.begin());
    }
    for (int gi = 0; gi < G.ngroup; ++gi) {
      FrontDev f{};
      f.off = G.gh[gi].fg_off;
      f.s = G.gh[gi].nc;
      fall.push_back(f);
      pbound = std::max(pbound, G.gh[gi].nc - khat[gi]);
    }
    pbound = ((pbound + kNB - 1) / kNB) * kNB;   // whole panels
    sweep_layout(sall, fall, true);
    G.fg = F.mem.get<T>(size_t(std::max<int64_t>(fg_all, 1)));
    G.info = F.mem.get<int>(G.ngroup);
    launch_fronts(pbound);
  }

  tm.mark("  launch IDs", l);
  F.flush_side(st);   // after the IDs
  tm.mark("  side work", l);
  std::vector<int32_t> kh(G.ngroup), ph(size_t(G.ngroup) * ncmax);
  LevelPivots piv;
  const size_t npiv = piv.count(F, l);
  int32_t* hk = static_cast<int32_t*>(F.host_stage((kh.size() + ph.size() + npiv) * 4));
  int32_t* hp = hk + kh.size();
  HIP_CHECK(hipMemcpyAsync(hk, G.kout, kh.size() * 4, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipMemcpyAsync(hp, G.perm, ph.size() * 4, hipMemcpyDeviceToHost, st));
  piv.queue(hp + ph.size(), st);
  HIP_CHECK(hipStreamSynchronize(st));
  std::copy(hk, hk + kh.size(), kh.begin());
  std::copy(hp, hp + ph.size(), ph.begin());
  piv.collect(hp + ph.size());
  tm.mark("  wait for IDs", l);
  check_input(F, st);
  piv.check(l, F.definite);
  // record skeletons; build the skeleton fronts
  int64_t fg_off = 0;
  G.gsel_h.clear();
  G.idx_h.clear();
  G.ff.clear();
  G.ncskel = 0;
  G.tel = G.rrows = G.krows = 0;
  int rmax = 0;
  for (int gi = 0; gi < G.ngroup; ++gi)
    if (kh[gi] < 0 || kh[gi] > G.gh[gi].nc) throw Error(HIFDE_EDEVICE, "ID returned an invalid rank");
  P.set_skeletons(l, kh.data(), ph.data(), size_t(ncmax));
  tm.mark("  set skeletons", l);
  if (!pre) {
    P.finish_groups(l);   // the planner's part: level l+1 can be planned now
    tm.mark("  finish groups", l);
    F.skel_job = std::async(std::launch::async, [&F, &G, &lev, kh = std::move(kh), l, st] {
      skeleton_fronts<T>(F, G, lev, kh, l, st);
    });
    return;
  }
  {
    size_t nidx = 0, nsk = 0;
    for (int gi = 0; gi < G.ngroup; ++gi)
      if (kh[gi] < G.gh[gi].nc) {
        nidx += size_t(G.gh[gi].nc);
        nsk += 1;
      }
    G.idx_h.reserve(nidx);
    G.ff.reserve(nsk);
    G.gsel_h.reserve(nsk);
  }
  // pre-launched skeleton fronts (their slots fixed before the IDs)
  for (int gi = 0; gi < G.ngroup; ++gi) {
    GroupDev& d = G.gh[gi];
    const int k = kh[gi];
    F.rank_groups += 1;
    F.rank_abs_err += std::abs(double(khat[gi]) - double(k));
    d.k = k;
    d.skel = (k < d.nc) ? 1 : 0;
    if (!d.skel) continue;
    G.tel += double(k) * (d.nc - k);
    G.rrows += d.nc - k;
    G.krows += k;
    rmax = std::max(rmax, d.nc - k);
    FrontDev f{};
    f.off = d.fg_off;
    f.s = d.nc;
    f.p = d.nc - k;
    f.idx = int64_t(G.idx_h.size());
    G.ff.push_back(f);
    fg_off += int64_t(d.nc) * d.nc;
    d.idx = int64_t(G.idx_h.size());
    const GroupRes& R = lev.res[gi];
    G.idx_h.insert(G.idx_h.end(), R.rd.begin(), R.rd.end());
    G.idx_h.insert(G.idx_h.end(), R.sk.begin(), R.sk.end());
    G.gsel_h.push_back(gi);
    G.ncskel = std::max(G.ncskel, int(d.nc));
  }
  tm.mark("  skeleton lists", l);
  P.finish_groups(l);
  tm.mark("  finish groups", l);
  G.nskel = int(G.gsel_h.size());
  G.groups = F.mem.upload(G.gh, st);
  {
    // a rank beyond the launched panels: eliminate every front again with
    // the actual bound (the IDs' choices are unchanged)
    if (rmax > pbound) {
      F.rebuckets += 1;
      launch_fronts(((rmax + kNB - 1) / kNB) * kNB);
    }
    // the sweeps see the skeletonized groups, in their pre-launch slots
    SweepSet& W = G.sw;
    W = SweepSet{};
    W.pk_elems = sall.pk_elems;
    W.pt_elems = sall.pt_elems;
    W.dv_elems = sall.dv_elems;
    for (int gi : G.gsel_h) {
      PackDev q = sall.ph[gi];
      q.p = G.gh[gi].nc - G.gh[gi].k;
      q.idx = G.gh[gi].idx;
      q.t_off = G.gh[gi].t_off;
      W.ph.push_back(q);
    }
    sweep_items(W, std::vector<int>(W.ph.size(), 0));
    upload_sweep(W, F.mem, st);
    if (G.nskel > 0) {
      G.idx = F.mem.upload(G.idx_h, st);
      G.gsel = F.mem.upload(G.gsel_h, st);
    }
    return;
  }
}

// TC: the type of the cell eliminations below the top; T: the type of the
// groups (IDs, skeletonization) and of the sweeps.  The top block is double.
template <typename TC, typename T>
static void run_factor(hifde_factor_s& F, hifde_tree_s* tree, hipStream_t st) {
  const int L = F.g.L;
  Planner& P = *F.planner;
  PhaseTimer tm;
  // the level-0 frontal matrices of a known tree are cleared first, so the
  // device does that while the host adopts the level-0 plan
  if (tree->l0 && tree->c0 && !F.plan_only) {
    F.cl[0].pool = F.mem.get<TC>(size_t(tree->c0->elems));
    if (tree->c0->smax >= kAsmWideFrom)   // (narrow assembly clears its own fronts)
      HIP_CHECK(hipMemsetAsync(F.cl[0].pool, 0, size_t(tree->c0->elems) * sizeof(TC), st));
  }
  // Level 0 and its groups depend on the geometry only: plan once per tree.
  if (!tree->l0) {
    P.plan_cells(0);
    P.plan_groups(0);
    tree->l0 = P.level0();
    tree->c0.reset();
    tree->g0.reset();
  } else {
    P.adopt_level0(tree->l0);
  }
  tm.mark("level-0 plan", 0);
  const auto t_start = std::chrono::steady_clock::now();
  for (int l = 0; l < L; ++l) {
    cells_level<TC, T>(F, tree, l, st);
    tm.mark("cells", l);
    groups_level<T>(F, tree, l, st);
    tm.mark("groups", l);
    if (l < HIFDE_MAX_LEVELS)
      F.stats.level_ms[l] = std::chrono::duration<double, std::milli>(
                                std::chrono::steady_clock::now() - t_start).count();
  }
  // the top block is bracketed by timing events (read after the final
  // synchronization below), after the last level's skeleton fronts are queued
  F.join_skel();
  hipEvent_t top_ev[2] = {nullptr, nullptr};
  if (!F.plan_only)
    for (hipEvent_t& e : top_ev) HIP_CHECK(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } ev_guard{top_ev};
  if (top_ev[0]) HIP_CHECK(hipEventRecord(top_ev[0], st));
  cells_level<double, double>(F, tree, L, st);
  if (top_ev[1]) HIP_CHECK(hipEventRecord(top_ev[1], st));
  F.flush_side(st);
  tm.mark("top", L);
  if (tm.on) {
    fprintf(stderr, "[hifde] uploads: %lld, %.1f KB, %.3f ms in the copy calls\n",
            static_cast<long long>(g_up_n.exchange(0)), double(g_up_bytes.exchange(0)) / 1024,
            double(g_up_ns.exchange(0)) * 1e-6);
  }
  if (F.plan_only) return;
  check_input(F, st);
  // pivot checks of every level at once: the flags are gathered on the
  // device and read back in one copy (one synchronization)
  {
    struct Part {
      const int* info;
      size_t n;
      const char* what;
      int l;
    };
    std::vector<Part> parts;
    size_t total = 0;
    for (int l = 0; l <= L; ++l) {
      const size_t nc = F.cl[l].st->fh.size();
      if (F.cl[l].info && nc > 0) parts.push_back({F.cl[l].info, nc, l == L ? "top block" : "cell", l});
      if (l < L && F.gl[l].info) {
        const size_t ni = F.presize ? size_t(F.gl[l].ngroup) : size_t(F.gl[l].nskel);
        if (ni > 0) parts.push_back({F.gl[l].info, ni, "group", l});
      }
    }
    for (const Part& q : parts) total += q.n;
    if (total > 0) {
      int* all = F.mem.get<int>(total);
      size_t at = 0;
      for (size_t b = 0; b < parts.size(); b += kFlagParts) {   // one launch per table
        FlagParts tab{};
        int64_t mx = 0;
        tab.off[0] = int64_t(at);
        for (size_t i = b; i < std::min(parts.size(), b + kFlagParts); ++i) {
          tab.p[tab.n] = parts[i].info;
          at += parts[i].n;
          tab.off[++tab.n] = int64_t(at);
          mx = std::max<int64_t>(mx, int64_t(parts[i].n));
        }
        const unsigned bx = unsigned(std::min<int64_t>(64, (mx + kThreads - 1) / kThreads));
        hipLaunchKernelGGL(k_gather_flags, dim3(bx, unsigned(tab.n)), dim3(kThreads), 0, st, tab,
                           all);
      }
      int* hp = static_cast<int*>(F.host_stage(total * sizeof(int)));
      HIP_CHECK(hipMemcpyAsync(hp, all, total * sizeof(int), hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      const std::vector<int> h(hp, hp + total);
      at = 0;
      for (const Part& q : parts) {
        report_info(std::vector<int>(h.begin() + at, h.begin() + at + q.n), q.what, q.l,
                    F.definite);
        at += q.n;
      }
    }
  }
  tm.mark("pivot checks", L);
  if (top_ev[1]) {
    HIP_CHECK(hipEventSynchronize(top_ev[1]));
    float ms = 0.0f;
    HIP_CHECK(hipEventElapsedTime(&ms, top_ev[0], top_ev[1]));
    F.stats.top_ms = ms;
  }
}

// The sweeps (and the packed apply form of every front below the top) are
// float under both mixed precisions.
static bool float_sweeps(const hifde_factor_s& F) { return F.prec != HIFDE_FP64; }

static void fill_stats(hifde_factor_s& F) {
  hifde_stats_t& s = F.stats;
  const Planner& P = *F.planner;
  s.precision = int32_t(F.prec);
  s.N = F.g.N;
  s.dim = F.g.dim;
  s.levels = F.g.L;
  double flops = 0.0, bytes = 0.0;
  int64_t mbytes = 0;
  const size_t esz = float_sweeps(F) ? 4 : 8;
  for (int l = 0; l <= F.g.L && l < HIFDE_MAX_LEVELS; ++l) {
    const Level& lev = P.level(l);
    s.cells[l] = int64_t(lev.cells().size());
    int mf = 0;
    const size_t e = (l == F.g.L) ? 8 : esz;
    for (const Cell& c : lev.cells()) {
      const double p = double(c.p.size()), q = double(c.q.size());
      flops += p * p * p / 3.0 + p * p * q + p * q * q;
      mf = std::max(mf, int(c.p.size() + c.q.size()));
      const double stored = p * (p + 1) / 2 + p * q;  // [L\D; W^T]
      bytes += 2.0 * stored * e;
      mbytes += int64_t(stored * e) + int64_t(4 * (p + q));
    }
    s.max_front[l] = mf;
    if (l == F.g.L) {
      s.top_size = lev.cells().empty() ? 0 : int64_t(lev.cells()[0].p.size());
      continue;
    }
    s.groups[l] = int64_t(lev.groups().size());
    int64_t in = 0, out = 0;
    for (size_t gi = 0; gi < lev.groups().size(); ++gi) {
      const Group& g = lev.groups()[gi];
      const GroupRes& R = lev.res[gi];
      in += int64_t(g.c.size());
      const double k = double(R.skel ? R.sk.size() : g.c.size());
      const double r = double(g.c.size()) - k;
      out += int64_t(k);
      if (R.skel) {
        flops += 2.0 * double(g.cN.size()) * double(g.c.size()) * k + r * r * r / 3.0 +
                 5.0 * k * r * r + 4.0 * k * k * r;
        const double stored = k * r + r * (r + 1) / 2 + k * r;  // T, [L_r\D_r; W_r^T]
        bytes += 2.0 * stored * esz;
        mbytes += int64_t(stored * esz) + int64_t(4 * g.c.size());
      }
    }
    s.skel_in[l] = in;
    s.skel_out[l] = out;
  }
  s.factor_flops = flops;
  s.solve_bytes = bytes;
  s.factor_bytes = mbytes;
  s.rank_groups = F.rank_groups;
  s.rank_mae = F.rank_groups > 0 ? F.rank_abs_err / double(F.rank_groups) : 0.0;
  s.rebuckets = F.rebuckets;
  s.skel_panels = F.skel_panels;
  s.tuned = F.tuned;
}

// ---------------------------------------------------------------------------
// Kernel timing: events around the launches of the profiled classes.
// ---------------------------------------------------------------------------
static void prof_collect(hifde_factor_s& F) {
  for (size_t i = 0; i < F.prof_used; ++i) {
    hifde_factor_s::ProfEvent& e = F.prof_ev[i];
    HIP_CHECK(hipEventSynchronize(e.b));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e.a, e.b));
    hifde_prof_t& acc = F.prof_acc[e.cls];
    acc.launches += 1;
    acc.ms += ms;
    acc.bytes += e.bytes;
    acc.flops += e.flops;
  }
  F.prof_used = 0;
}

template <class Launch>
static void timed(hifde_factor_s& F, int cls, int level, double bytes, double flops,
                  hipStream_t st, Launch&& launch) {
  if (!((F.prof_mask >> cls) & 1u) || (F.prof_level >= 0 && F.prof_level != level)) {
    launch();
    return;
  }
  if (F.prof_used == 4096) prof_collect(F);
  if (F.prof_used == F.prof_ev.size()) {
    hifde_factor_s::ProfEvent e;
    HIP_CHECK(hipEventCreate(&e.a));
    HIP_CHECK(hipEventCreate(&e.b));
    F.prof_ev.push_back(e);
  }
  hifde_factor_s::ProfEvent& e = F.prof_ev[F.prof_used++];
  e.cls = cls;
  e.bytes = bytes;
  e.flops = flops;
  HIP_CHECK(hipEventRecord(e.a, st));
  launch();
  HIP_CHECK(hipEventRecord(e.b, st));
}

// Algorithmic work of one sweep launch over the fronts of color c (-1: all)
// of a set: the apply-form elements p(p+1)/2 + (s-p)p (D^-1 included) are
// read once, the unknown lists once, and the vector rows as the step
// formulas touch them (up: read s rows, write s rows; down: read s rows,
// write p rows).
struct Work {
  double bytes, flops;
};
static Work sweep_work(const SweepSet& S, int color, bool up, int nrhs, size_t esz, size_t xsz) {
  double fac = 0, sr = 0, pr = 0;
  for (int c = 0; c < 2; ++c)
    if (color < 0 || color == c) {
      fac += S.fac[c];
      sr += S.srows[c];
      pr += S.prows[c];
    }
  if (up) return {fac * esz + sr * 4 + 2 * sr * nrhs * xsz, 2.0 * nrhs * fac};
  return {(fac - pr) * esz + sr * 4 + (sr + pr) * nrhs * xsz, 2.0 * nrhs * (fac - pr)};
}
// Interpolation step of a level's groups: T (kr elements) once, the
// skeleton (up) or redundant (down) rows read, the other rows updated.
static Work interp_work(const GroupLevel& G, bool up, int nrhs, size_t esz, size_t xsz) {
  const double rd = up ? G.krows : G.rrows, rw = up ? G.rrows : G.krows;
  return {G.tel * esz + (G.rrows + G.krows) * 4 + (rd + 2 * rw) * nrhs * xsz,
          2.0 * nrhs * G.tel};
}

// Launch shape of a sweep: NT = 16-column tiles of right-hand sides per
// work-group, the LDS rows of one staging chunk (at most 32 KiB), the grid.
constexpr int kSwLdsCap = 32 * 1024;
struct SweepShape {
  int NT, nch, kch;
  size_t lds;
  unsigned grid;
};
template <typename T>
static SweepShape sweep_shape(int nitems, int nrhs, int krows) {
  SweepShape g{};
  g.NT = nrhs <= 16 ? 1 : nrhs <= 32 ? 2 : 4;
  g.nch = (nrhs + 16 * g.NT - 1) / (16 * g.NT);
  const int stride = sweep_stride(g.NT);
  const int cap = (kSwLdsCap / (stride * int(sizeof(T)))) & ~15;
  g.kch = std::min(cap, std::max(16, (krows + 15) & ~15));
  g.lds = size_t(g.kch) * stride * sizeof(T);
  const int64_t grid = int64_t(8) * ((nitems + 7) / 8) * g.nch;
  if (grid > INT32_MAX) throw Error(HIFDE_EINVAL, "sweep grid too large");
  g.grid = unsigned(grid);
  return g;
}

// Output chunks of the largest group's interpolation step.
static unsigned interp_chunks(const GroupLevel& G, int nrhs, bool up) {
  int64_t m = 1;
  for (int gi : G.gsel_h) {
    const GroupDev& d = G.gh[gi];
    m = std::max<int64_t>(m, int64_t(up ? d.nc - d.k : d.k) * nrhs);
  }
  const int64_t ch = (m + kInterpChunk - 1) / kInterpChunk;
  if (ch > 65535) throw Error(HIFDE_EINVAL, "interpolation step too large for its grid");
  return unsigned(ch);
}

// Whole-front steps (one work-group per front and column chunk) when a
// launch has at least kSwWholeMin of them and the staged rows fit
// kSwWholeLds bytes of LDS.
constexpr int kSwWholeLds = 40 * 1024;
static int sweep_whole_min() {
  static const int v = [] {
    const char* e = std::getenv("HIFDE_SWEEP_WHOLE_MIN");
    return e ? std::max(1, std::atoi(e)) : 1024;
  }();
  return v;
}
template <typename T>
static bool sweep_whole(int nfronts, int nrhs, int rows, SweepShape* g, bool any_count = false) {
  const int NT = nrhs <= 16 ? 1 : nrhs <= 32 ? 2 : 4;
  const int nch = (nrhs + 16 * NT - 1) / (16 * NT);
  const size_t lds = size_t(rows) * sweep_stride(NT) * sizeof(T);
  if (nfronts == 0 || lds > size_t(kSwWholeLds)) return false;
  if (!any_count && int64_t(nfronts) * nch < sweep_whole_min()) return false;
  g->NT = NT;
  g->nch = nch;
  g->kch = rows;
  g->lds = lds;
  g->grid = unsigned(int64_t(8) * ((nfronts + 7) / 8) * nch);
  return true;
}

// One upward sweep launch over the fronts of color c of S.  With `tpool`
// (a group level) only the whole-front form with the interpolation fused is
// tried: returns false when it does not fit, and the caller runs the
// interpolation and the row-tile form instead.
template <typename T, typename TX>
static bool sweep_up(hifde_factor_s& F, int cls, int level, const SweepSet& S, int c,
                     const void* pk, const void* dinv, const int32_t* idx, TX* X, TX* Z, int nrhs,
                     hipStream_t st, const void* tpool = nullptr, Work extra = Work{0, 0}) {
  const int n = int(S.up_h[c].size());
  if (n == 0) return true;
  SweepShape g{};
  const int nf = int(S.upf_h[c].size());
  const bool whole = !F.row_tiles && sweep_whole<T>(nf, nrhs, S.kdown, &g, tpool != nullptr);
  if (tpool && !whole) return false;
  if (!whole) g = sweep_shape<T>(n, nrhs, S.kup);
  Work w = F.prof_mask ? sweep_work(S, c, true, nrhs, sizeof(T), sizeof(TX)) : Work{0, 0};
  w.bytes += extra.bytes;
  w.flops += extra.flops;
  const T* P = static_cast<const T*>(pk);
  const T* Dv = static_cast<const T*>(dinv);
  const T* Tp = static_cast<const T*>(tpool);
  const bool vec = nrhs % int(16 / sizeof(TX)) == 0;
  const int pcls = !whole || cls != HIFDE_PROF_SWEEP_UP ? cls
                   : tpool ? HIFDE_PROF_GROUP_UP : HIFDE_PROF_SWEEP_UP_WHOLE;
  timed(F, pcls, level, w.bytes, w.flops, st, [&] {
#define HIFDE_UP(NTV, VV)                                                                         \
  if (whole && tpool)                                                                             \
    hipLaunchKernelGGL((k_sweep_up_f<T, TX, NTV, VV, true>), dim3(g.grid), dim3(kThreads), g.lds, \
                       st, S.packs, S.upf[c], nf, g.nch, P, Dv, idx, X, Z, nrhs, Tp);             \
  else if (whole)                                                                                 \
    hipLaunchKernelGGL((k_sweep_up_f<T, TX, NTV, VV, false>), dim3(g.grid), dim3(kThreads), g.lds, \
                       st, S.packs, S.upf[c], nf, g.nch, P, Dv, idx, X, Z, nrhs, Tp);             \
  else                                                                                          \
    hipLaunchKernelGGL((k_sweep_up<T, TX, NTV, VV>), dim3(g.grid), dim3(kThreads), g.lds, st,   \
                       S.packs, S.up[c], n, g.nch, P, Dv, idx, X, Z, nrhs, g.kch)
    if (vec) {
      if (g.NT == 1) HIFDE_UP(1, true); else if (g.NT == 2) HIFDE_UP(2, true); else HIFDE_UP(4, true);
    } else {
      if (g.NT == 1) HIFDE_UP(1, false); else if (g.NT == 2) HIFDE_UP(2, false); else HIFDE_UP(4, false);
    }
#undef HIFDE_UP
  });
  return true;
}

// The upward step of both colors of a cell level in one launch
// (k_sweep_up_c) and the addition of the x_q contributions
// (k_contrib_add).  Returns false when the level has no contribution plan
// or the whole-front form does not apply; the caller then launches the two
// colors.
template <typename T, typename TX>
static bool sweep_up_one(hifde_factor_s& F, int level, const SweepSet& S, const void* pk,
                         const void* dinv, const int32_t* idx, TX* X, TX* Z, int nrhs,
                         hipStream_t st) {
  if (S.upc_h.empty() || F.row_tiles) return false;
  const int nf = int(S.upc_h.size()), nq = int(S.qunk_h.size());
  if (int64_t(nq) * nrhs >= INT32_MAX) return false;
  SweepShape g{};
  if (!sweep_whole<T>(nf, nrhs, S.kpf, &g)) return false;
  if (F.C.bytes < size_t(S.cq_rows) * size_t(nrhs) * sizeof(T))
    throw Error(HIFDE_ESTATE, "contribution buffer too small");
  T* C = F.C.as<T>();
  const size_t esz = sizeof(T), xsz = sizeof(TX);
  Work w{0, 0};
  if (F.prof_mask) {
    // the stored factor read once and each front's p and q vector rows once
    // per right-hand side (one upward pass of the level-0 cells)
    const double fac = S.fac[0] + S.fac[1], pr = S.prows[0] + S.prows[1];
    const double qr = double(S.cq_rows);
    w = {fac * esz + (pr + qr) * xsz * nrhs, 2.0 * nrhs * fac};
  }
  const T* P = static_cast<const T*>(pk);
  const T* Dv = static_cast<const T*>(dinv);
  const bool vec = nrhs % int(16 / sizeof(TX)) == 0;
  if (F.upc_part != 2)
  timed(F, HIFDE_PROF_SWEEP_UP_ONE, level, w.bytes, w.flops, st, [&] {
#define HIFDE_UPC(NTV, VV)                                                                   \
  hipLaunchKernelGGL((k_sweep_up_c<T, TX, NTV, VV>), dim3(g.grid), dim3(kThreads), g.lds, st, \
                     S.packs, S.upc, nf, g.nch, P, Dv, idx, X, Z, C, nrhs)
    if (vec) {
      if (g.NT == 1) HIFDE_UPC(1, true); else if (g.NT == 2) HIFDE_UPC(2, true); else HIFDE_UPC(4, true);
    } else {
      if (g.NT == 1) HIFDE_UPC(1, false); else if (g.NT == 2) HIFDE_UPC(2, false); else HIFDE_UPC(4, false);
    }
#undef HIFDE_UPC
  });
  if (F.upc_part == 1) return true;
  const double nc = double(S.qsrc_h.size());
  const Work wa = F.prof_mask ? Work{double(nq) * nrhs * 2 * xsz + nc * nrhs * esz +
                                         double(nq) * 8 + nc * 4,
                                     double(nc) * nrhs}
                              : Work{0, 0};
  const unsigned blocks = unsigned((int64_t(nq) * nrhs + kThreads - 1) / kThreads);
  timed(F, HIFDE_PROF_CONTRIB_ADD, level, wa.bytes, wa.flops, st, [&] {
    hipLaunchKernelGGL((k_contrib_add<T, TX>), dim3(blocks), dim3(kThreads), 0, st, S.qunk,
                       S.qptr, S.qsrc, nq, static_cast<const T*>(C), X, nrhs);
  });
  return true;
}

// One downward sweep launch; `tpool` as in sweep_up (the interpolation
// follows the step, in the same launch).
template <typename T, typename TX>
static bool sweep_down(hifde_factor_s& F, int cls, int level, const SweepSet& S, const void* pt,
                       const int32_t* idx, TX* X, const TX* Z, int nrhs, hipStream_t st,
                       const void* tpool = nullptr, Work extra = Work{0, 0}) {
  const int n = int(S.down_h.size());
  if (n == 0) return true;
  SweepShape g{};
  const int nf = int(S.downf_h.size());
  const int rows = S.kdown + (tpool ? S.kpf : 0);   // staged rows (+ new x_r)
  const bool whole = !F.row_tiles && sweep_whole<T>(nf, nrhs, rows, &g, tpool != nullptr);
  if (tpool && !whole) return false;
  if (!whole) g = sweep_shape<T>(n, nrhs, S.kdown);
  Work w = F.prof_mask ? sweep_work(S, -1, false, nrhs, sizeof(T), sizeof(TX)) : Work{0, 0};
  w.bytes += extra.bytes;
  w.flops += extra.flops;
  const T* P = static_cast<const T*>(pt);
  const T* Tp = static_cast<const T*>(tpool);
  const bool vec = nrhs % int(16 / sizeof(TX)) == 0;
  const int pcls = !whole || cls != HIFDE_PROF_SWEEP_DOWN ? cls
                   : tpool ? HIFDE_PROF_GROUP_DOWN : HIFDE_PROF_SWEEP_DOWN_WHOLE;
  timed(F, pcls, level, w.bytes, w.flops, st, [&] {
#define HIFDE_DN(NTV, VV)                                                                           \
  if (whole && tpool)                                                                               \
    hipLaunchKernelGGL((k_sweep_down_f<T, TX, NTV, VV, true>), dim3(g.grid), dim3(kThreads), g.lds, \
                       st, S.packs, S.downf, nf, g.nch, P, idx, X, Z, nrhs, Tp);                    \
  else if (whole)                                                                                   \
    hipLaunchKernelGGL((k_sweep_down_f<T, TX, NTV, VV, false>), dim3(g.grid), dim3(kThreads),      \
                       g.lds, st, S.packs, S.downf, nf, g.nch, P, idx, X, Z, nrhs, Tp);            \
  else                                                                                            \
    hipLaunchKernelGGL((k_sweep_down<T, TX, NTV, VV>), dim3(g.grid), dim3(kThreads), g.lds, st,   \
                       S.packs, S.down, n, g.nch, P, idx, X, Z, nrhs, g.kch)
    if (vec) {
      if (g.NT == 1) HIFDE_DN(1, true); else if (g.NT == 2) HIFDE_DN(2, true); else HIFDE_DN(4, true);
    } else {
      if (g.NT == 1) HIFDE_DN(1, false); else if (g.NT == 2) HIFDE_DN(2, false); else HIFDE_DN(4, false);
    }
#undef HIFDE_DN
  });
  return true;
}

// ---------------------------------------------------------------------------
// F^-1 application on unknown-major vectors X (type TX); Z (same size) holds
// the values z_p of the eliminated unknowns between the two sweeps.
// ---------------------------------------------------------------------------
template <typename T, typename TX>
static void apply_inverse(hifde_factor_s& F, TX* X, TX* Z, int nrhs, hipStream_t st) {
  const int L = F.g.L;
  const size_t esz = sizeof(T), xsz = sizeof(TX);
  for (int l = 0; l < L; ++l) {
    CellLevel& C = F.cl[l];
    const CellStatic& S = *C.st;
    if (!sweep_up_one<T, TX>(F, l, S.sw, C.pk, C.dinv, S.idx, X, Z, nrhs, st))
      for (int color = 0; color < 2; ++color)
        sweep_up<T, TX>(F, HIFDE_PROF_SWEEP_UP, l, S.sw, color, C.pk, C.dinv, S.idx, X, Z, nrhs,
                        st);
    GroupLevel& G = F.gl[l];
    if (G.nskel > 0) {
      // interpolation and elimination of ř in one launch when the fronts fit
      const Work w = F.prof_mask ? interp_work(G, true, nrhs, esz, xsz) : Work{0, 0};
      if (!sweep_up<T, TX>(F, HIFDE_PROF_SWEEP_UP, l, G.sw, 0, G.pk, G.dinv, G.idx, X, Z, nrhs,
                           st, G.tpool, w)) {
        timed(F, HIFDE_PROF_INTERP, l, w.bytes, w.flops, st, [&] {
          hipLaunchKernelGGL((k_interp_up<T, TX>), dim3(G.nskel, interp_chunks(G, nrhs, true)),
                             dim3(kThreads), 0, st, G.groups, G.gsel,
                             static_cast<const T*>(G.tpool), G.idx, X, nrhs);
        });
        sweep_up<T, TX>(F, HIFDE_PROF_SWEEP_UP, l, G.sw, 0, G.pk, G.dinv, G.idx, X, Z, nrhs, st);
      }
    }
  }
  CellLevel& top = F.cl[L];
  sweep_up<double, TX>(F, HIFDE_PROF_TOP, L, top.st->sw, 0, top.pk, top.dinv, top.st->idx, X, Z,
                       nrhs, st);
  sweep_down<double, TX>(F, HIFDE_PROF_TOP, L, top.st->sw, top.pt, top.st->idx, X, Z, nrhs, st);
  for (int l = L - 1; l >= 0; --l) {
    GroupLevel& G = F.gl[l];
    if (G.nskel > 0) {
      const Work w = F.prof_mask ? interp_work(G, false, nrhs, esz, xsz) : Work{0, 0};
      if (!sweep_down<T, TX>(F, HIFDE_PROF_SWEEP_DOWN, l, G.sw, G.pt, G.idx, X, Z, nrhs, st,
                             G.tpool, w)) {
        sweep_down<T, TX>(F, HIFDE_PROF_SWEEP_DOWN, l, G.sw, G.pt, G.idx, X, Z, nrhs, st);
        timed(F, HIFDE_PROF_INTERP, l, w.bytes, w.flops, st, [&] {
          hipLaunchKernelGGL((k_interp_down<T, TX>), dim3(G.nskel, interp_chunks(G, nrhs, false)),
                             dim3(kThreads), 0, st, G.groups, G.gsel,
                             static_cast<const T*>(G.tpool), G.idx, X, nrhs);
        });
      }
    }
    CellLevel& C = F.cl[l];
    sweep_down<T, TX>(F, HIFDE_PROF_SWEEP_DOWN, l, C.st->sw, C.pt, C.st->idx, X, Z, nrhs, st);
  }
  HIP_CHECK(hipGetLastError());
}

// F^-1 application through a HIP graph: the launches of one application
// (fixed buffers, fixed right-hand-side count) are captured once on a
// private stream and replayed on the caller's stream.  Timed launches
// (hifde_profile: HIP reports no durations for events recorded inside a
// graph) and HIFDE_NO_GRAPH use direct launches.  The one-launch level-0
// upward sweep, when the application starts with it, is launched directly
// before the graph (also when it alone is timed).
template <typename T, typename TX>
static void apply_inverse_g(hifde_factor_s& F, TX* X, TX* Z, int nrhs, hipStream_t st) {
  // The application's first kernel, the one-launch level-0 upward sweep,
  // runs directly and the rest from a graph captured without it: the graph's
  // launch then overlaps that kernel instead of delaying the application
  // (and the kernel can be timed).
  const bool first_only = F.prof_mask == 0 || F.prof_mask == (1u << HIFDE_PROF_SWEEP_UP_ONE);
  if (!F.use_graph || !first_only) {
    apply_inverse<T, TX>(F, X, Z, nrhs, st);
    return;
  }
  int part = 0;
  if (first_only) {
    CellLevel& C0 = F.cl[0];
    const CellStatic& S0 = *C0.st;
    F.upc_part = 1;
    bool did = false;
    try {
      did = F.g.L > 0 &&
            sweep_up_one<T, TX>(F, 0, S0.sw, C0.pk, C0.dinv, S0.idx, X, Z, nrhs, st);
    } catch (...) {
      F.upc_part = 0;
      throw;
    }
    F.upc_part = 0;
    if (did) part = 2;   // else no one-launch form: the whole application from the graph
  }
  if (!(F.gexec && F.g_nrhs == nrhs && F.g_x == X && F.g_z == Z && F.g_c == F.C.p &&
        F.g_part == part)) {
    if (F.gexec) {
      HIP_CHECK(hipGraphExecDestroy(F.gexec));
      F.gexec = nullptr;
    }
    if (!F.cap) F.cap = StreamCache::get().take();
    HIP_CHECK(hipStreamBeginCapture(F.cap, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    const uint32_t mask = F.prof_mask;
    F.prof_mask = 0;   // (nothing timed inside the graph)
    F.upc_part = part;
    try {
      apply_inverse<T, TX>(F, X, Z, nrhs, F.cap);
    } catch (...) {
      F.prof_mask = mask;
      F.upc_part = 0;
      (void)hipStreamEndCapture(F.cap, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    F.prof_mask = mask;
    F.upc_part = 0;
    HIP_CHECK(hipStreamEndCapture(F.cap, &g));
    hipError_t e = hipGraphInstantiate(&F.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      F.gexec = nullptr;
      HIP_CHECK(e);
    }
    F.g_nrhs = nrhs;
    F.g_x = X;
    F.g_z = Z;
    F.g_c = F.C.p;
    F.g_part = part;
  }
  HIP_CHECK(hipGraphLaunch(F.gexec, st));
}

static void ensure_X(hifde_factor_s& F, int64_t nrhs) {
  const size_t need = size_t(F.g.N) * size_t(nrhs) * 8;
  if (F.X.bytes < need) F.X.alloc(need);
  if (F.Z.bytes < need) F.Z.alloc(need);
  const int64_t rows = F.cl.empty() || !F.cl[0].st ? 0 : F.cl[0].st->sw.cq_rows;
  const size_t cneed = size_t(rows) * size_t(nrhs) * 8;
  if (cneed > 0 && F.C.bytes < cneed) F.C.alloc(cneed);
}


// Blocks of a PCG pass: one full round of the device at the kernel's
// occupancy (its register count decides how many work-groups a CU holds;
// a second, partial round would leave most of the device idle), a multiple
// of 8 for the XCD-major block ranges, at most kPcgBlocks.
static unsigned pcg_blocks(const void* kernel) {
  int per_cu = 0, dev = 0, cus = 0;
  HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0));
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t nb = (int64_t(std::max(per_cu, 1)) * std::max(cus, 1)) / 8 * 8;
  return unsigned(std::min<int64_t>(std::max<int64_t>(nb, 8), kPcgBlocks));
}

// Conjugate gradients preconditioned by F^-1 (Section 5), one independent
// iteration per column, all vectors unknown-major in double; TR is the type
// of the preconditioner's vectors (float: flexible beta).  Returns whether
// every column reached tol.
template <typename TR, int W, int DIM>
static bool run_pcg_w(hifde_factor_s& F, int64_t nrhs, const double* f, int64_t ldf, double* u,
                      int64_t ldu, double tol, int maxit, int* iters, double* relres,
                      hipStream_t st) {
  using TP = typename std::conditional<sizeof(TR) == 4, float, double>::type;
  const int64_t N = F.g.N, n = N * nrhs;
  const int nr = int(nrhs);
  const int flexible = sizeof(TR) == 4 ? 1 : 0;
  // vectors: x r and two p buffers (double), two partial sets, scalars
  const size_t vbytes = size_t(n) * 8;
  const size_t pbytes = size_t(kPcgBlocks) * 2 * nr * 8;
  if (F.pcg_rhs != nrhs) {
    F.pcg.alloc(vbytes * 4 + pbytes * 2 + size_t(nr) * 8 * 8 + size_t(nr) * 4);
    F.pcg_rhs = nrhs;
  }
  ensure_X(F, nrhs);
  TR* rc = F.X.as<TR>();          // r in the preconditioner's type, turned into z by F^-1
  TR* Zs = F.Z.as<TR>();
  char* base = F.pcg.as<char>();
  double* x = reinterpret_cast<double*>(base);
  double* r = x + n;
  double* pa = r + n;              // p of the last iteration
  double* pb = pa + n;             // p of this one
  double* px = pb + n;             // partials of k_pcg_xr
  double* pz = px + size_t(kPcgBlocks) * 2 * nr;   // partials of k_pcg_ap / k_pcg_rz
  double* sc = pz + size_t(kPcgBlocks) * 2 * nr;
  double* rz = sc;
  double* alpha = sc + nr;
  double* beta = sc + 2 * nr;
  double* d1 = sc + 3 * nr;
  int* live = reinterpret_cast<int*>(sc + 8 * nr);
  const unsigned nb_ap = pcg_blocks(reinterpret_cast<const void*>(&k_pcg_ap<TR, W, DIM>));
  const unsigned nb_xr = pcg_blocks(reinterpret_cast<const void*>(&k_pcg_xr<TR, W, DIM>));
  const unsigned nb_rz = pcg_blocks(reinterpret_cast<const void*>(&k_pcg_rz<TR, W>));
  const int64_t side = F.g.n;
  const DivN dn = make_divn(uint32_t(side));
  const double* diag = F.diag.as<double>();
  const double* offd = F.offd.as<double>();

  HIP_CHECK(hipMemsetAsync(pa, 0, vbytes, st));
  HIP_CHECK(hipMemsetAsync(alpha, 0, size_t(nr) * 8, st));
  HIP_CHECK(hipMemsetAsync(rz, 0, size_t(nr) * 8, st));
  // r = f, the preconditioner's copy of r, x = 0 and ||f||^2
  const unsigned nb_st = pcg_blocks(reinterpret_cast<const void*>(&k_pcg_start<TR, W>));
  hipLaunchKernelGGL((k_pcg_start<TR, W>), dim3(nb_st), dim3(kThreads), 0, st, N, nr, f, ldf, x, r,
                     rc, px);
  hipLaunchKernelGGL(k_reduce_sum, dim3(nr), dim3(kThreads), 0, st, int(nb_st), nr, 0, px, d1);
  std::vector<int> liveh(nr, 1), itsh(nr, 0);
  std::vector<double> fh(nr), h1(nr);
  double* hd = static_cast<double*>(F.host_stage(size_t(nr) * 8));   // pinned read-backs
  HIP_CHECK(hipMemcpyAsync(hd, d1, nr * 8, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  std::copy(hd, hd + nr, fh.begin());
  for (int c = 0; c < nr; ++c) {
    fh[c] = std::sqrt(fh[c]);
    if (fh[c] == 0.0) liveh[c] = 0;
  }
  HIP_CHECK(hipMemcpyAsync(live, liveh.data(), nr * 4, hipMemcpyHostToDevice, st));
  apply_inverse_g<TP, TR>(F, rc, Zs, nr, st);
  // rz = r.z, beta = 0 (rz was 0)
  hipLaunchKernelGGL((k_pcg_rz<TR, W>), dim3(nb_rz), dim3(kThreads), 0, st, N, nr, rc, r, pz);
  hipLaunchKernelGGL(k_reduce_beta, dim3(nr), dim3(kThreads), 0, st, int(nb_rz), int(nb_xr), nr,
                     pz, px, 0, rz, live, beta);
  int it = 0;
  while (it < maxit) {
    bool any = false;
    for (int c = 0; c < nr; ++c) any = any || liveh[c];
    if (!any) break;
    ++it;
    hipLaunchKernelGGL((k_pcg_ap<TR, W, DIM>), dim3(nb_ap), dim3(kThreads), 0, st, N, nr, dn,
                       diag, offd, beta, rc, pa, pb, pz);
    hipLaunchKernelGGL(k_reduce_alpha, dim3(nr), dim3(kThreads), 0, st, int(nb_ap), nr, pz, rz,
                       live, alpha);
    hipLaunchKernelGGL((k_pcg_xr<TR, W, DIM>), dim3(nb_xr), dim3(kThreads), 0, st, N, nr, dn,
                       diag, offd, alpha, pb, x, r, rc, flexible, px);
    hipLaunchKernelGGL(k_reduce_sum, dim3(nr), dim3(kThreads), 0, st, int(nb_xr), nr, 0, px, d1);
    std::swap(pa, pb);
    HIP_CHECK(hipMemcpyAsync(hd, d1, nr * 8, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    std::copy(hd, hd + nr, h1.begin());
    bool changed = false, anyl = false;
    for (int c = 0; c < nr; ++c) {
      if (!liveh[c]) continue;
      itsh[c] = it;
      if (std::sqrt(h1[c]) <= tol * fh[c]) {
        liveh[c] = 0;
        changed = true;
      }
      anyl = anyl || liveh[c];
    }
    if (changed) HIP_CHECK(hipMemcpyAsync(live, liveh.data(), nr * 4, hipMemcpyHostToDevice, st));
    if (!anyl || it == maxit) break;
    apply_inverse_g<TP, TR>(F, rc, Zs, nr, st);
    hipLaunchKernelGGL((k_pcg_rz<TR, W>), dim3(nb_rz), dim3(kThreads), 0, st, N, nr, rc, r, pz);
    hipLaunchKernelGGL(k_reduce_beta, dim3(nr), dim3(kThreads), 0, st, int(nb_rz), int(nb_xr), nr,
                       pz, px, flexible, rz, live, beta);
  }
  // true residuals ||f - A x|| and u = x, in one pass over x and f
  const unsigned nb_tr =
      pcg_blocks(reinterpret_cast<const void*>(&k_pcg_true_resid<W, DIM>));
  hipLaunchKernelGGL((k_pcg_true_resid<W, DIM>), dim3(nb_tr), dim3(kThreads), 0, st, N, nr, dn,
                     diag, offd, x, f, ldf, u, ldu, px);
  hipLaunchKernelGGL(k_reduce_sum, dim3(nr), dim3(kThreads), 0, st, int(nb_tr), nr, 0, px, d1);
  HIP_CHECK(hipMemcpyAsync(hd, d1, nr * 8, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));
  std::copy(hd, hd + nr, h1.begin());
  bool converged = true;
  for (int c = 0; c < nr; ++c) {
    iters[c] = itsh[c];
    relres[c] = fh[c] > 0 ? std::sqrt(h1[c]) / fh[c] : 0.0;
    if (liveh[c]) converged = false;
  }
  return converged;
}

template <typename TR>
static bool run_pcg(hifde_factor_s& F, int64_t nrhs, const double* f, int64_t ldf, double* u,
                    int64_t ldu, double tol, int maxit, int* iters, double* relres,
                    hipStream_t st) {
  const bool even = nrhs % 2 == 0;
  if (F.g.dim == 2)
    return even ? run_pcg_w<TR, 2, 2>(F, nrhs, f, ldf, u, ldu, tol, maxit, iters, relres, st)
                : run_pcg_w<TR, 1, 2>(F, nrhs, f, ldf, u, ldu, tol, maxit, iters, relres, st);
  return even ? run_pcg_w<TR, 2, 3>(F, nrhs, f, ldf, u, ldu, tol, maxit, iters, relres, st)
              : run_pcg_w<TR, 1, 3>(F, nrhs, f, ldf, u, ldu, tol, maxit, iters, relres, st);
}

// GMRES with F^-1 as right preconditioner (Section 5), restarted every m
// steps, one independent iteration per column, vectors unknown-major in
// double; TR is the type of the preconditioner's vectors.  The basis and
// the inner products stay on the device; the host reads each step's
// Hessenberg column (m + 2 values per column at most) and applies the
// Givens rotations.  All live columns step together: a column that has
// converged gets zero basis vectors (its h is 0), so its later steps add
// nothing.  Returns whether every column reached tol.
template <typename TR>
static bool run_gmres(hifde_factor_s& F, int64_t nrhs, const double* f, int64_t ldf, double* u,
                      int64_t ldu, double tol, int m, int maxit, int* iters, double* relres,
                      hipStream_t st) {
  using TP = typename std::conditional<sizeof(TR) == 4, float, double>::type;
  const int64_t N = F.g.N, n = N * nrhs;
  const int nr = int(nrhs);
  const size_t need = (size_t(m) + 3) * size_t(n) * 8 + size_t(m) * size_t(n) * sizeof(TR) +
                      (size_t(kGmBlocks) * 2 + size_t(m) * 2 + 3) * size_t(nr) * 8;
  if (F.gm.bytes < need) F.gm.alloc(need);
  ensure_X(F, nrhs);
  TR* X = F.X.as<TR>();
  TR* Zs = F.Z.as<TR>();
  double* V = F.gm.as<double>();                 // v_0 .. v_m
  double* w = V + size_t(m + 1) * n;
  double* x = w + n;
  double* part = x + n;                          // kGmBlocks x 2 x nr
  double* h = part + size_t(kGmBlocks) * 2 * nr; // (m + 2) x nr
  double* den = h + size_t(m + 2) * nr;          // nr
  double* Yd = den + nr;                         // m x nr
  TR* Zk = reinterpret_cast<TR*>(Yd + size_t(m) * nr);   // z_0 .. z_{m-1}
  const unsigned nb = unsigned(std::min<int64_t>(kGmBlocks, std::max<int64_t>(1, nblk(n))));
  const unsigned ne = nblk(n);
  const int dim = F.g.dim;
  const int64_t side = F.g.n;
  const double* diag = F.diag.as<double>();
  const double* offd = F.offd.as<double>();
  auto mgs = [&](const double* coef, const double* vprev, const double* v, double* out) {
    hipLaunchKernelGGL(k_gm_mgs, dim3(nb), dim3(kThreads), 0, st, N, nr, coef, vprev, v, w, part);
    hipLaunchKernelGGL(k_reduce_sum, dim3(nr), dim3(kThreads), 0, st, int(nb), nr, 0, part, out);
  };
  double* hd = static_cast<double*>(F.host_stage(size_t(m + 2) * nr * 8));   // pinned
  auto read_h = [&](std::vector<double>& hh, int rows) {
    HIP_CHECK(hipMemcpyAsync(hd, h, size_t(rows) * nr * 8, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    std::copy(hd, hd + size_t(rows) * nr, hh.begin());
  };
  const size_t ldh = size_t(m) + 1;              // H of column c: Hs[c][i + j ldh]
  std::vector<double> hh(size_t(m + 2) * nr), nf(nr, 0.0), denh(nr), Yh(size_t(m) * nr);
  std::vector<double> Hs(ldh * m * nr), cs(size_t(m) * nr), sn(size_t(m) * nr), g(ldh * nr);
  std::vector<int> live(nr, 1), act(nr, 0), kd(nr, 0), its(nr, 0);
  HIP_CHECK(hipMemsetAsync(x, 0, size_t(n) * 8, st));
  int it = 0;
  for (bool first = true;; first = false) {
    // r = f - A x (the true residual) into w, and its norm
    hipLaunchKernelGGL(k_gm_residual, dim3(ne), dim3(kThreads), 0, st, N, nr, dim, side, diag,
                       offd, f, ldf, x, w);
    mgs(nullptr, nullptr, nullptr, h);
    read_h(hh, 1);
    bool any = false;
    for (int c = 0; c < nr; ++c) {
      const double beta = std::sqrt(hh[c]);
      if (first) {
        nf[c] = beta;
        if (beta == 0.0) live[c] = 0;
      }
      if (live[c] && beta <= tol * nf[c]) live[c] = 0;
      act[c] = live[c];
      kd[c] = 0;
      denh[c] = act[c] ? beta : 0.0;
      g[c * ldh] = beta;
      any = any || act[c];
    }
    if (!any || it >= maxit) break;   // hh holds ||f - A x||^2 of the final x
    HIP_CHECK(hipMemcpyAsync(den, denh.data(), size_t(nr) * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_gm_div, dim3(ne), dim3(kThreads), 0, st, n, nr, den, w, V);
    for (int k = 0; k < m; ++k) {
      ++it;
      // w = A z_k, z_k = F^-1 v_k (kept for the update of x)
      hipLaunchKernelGGL((k_gm_convert<TR>), dim3(ne), dim3(kThreads), 0, st, n,
                         V + size_t(k) * n, X);
      apply_inverse_g<TP, TR>(F, X, Zs, nr, st);
      hipLaunchKernelGGL((k_gm_matvec<TR>), dim3(ne), dim3(kThreads), 0, st, N, nr, dim, side,
                         diag, offd, X, Zk + size_t(k) * n, w);
      // modified Gram-Schmidt: h_ik = v_i . w, w -= h_ik v_i in turn, then
      // ||w||^2
      for (int i = 0; i <= k; ++i)
        mgs(i ? h + size_t(i - 1) * nr : nullptr, i ? V + size_t(i - 1) * n : nullptr,
            V + size_t(i) * n, h + size_t(i) * nr);
      mgs(h + size_t(k) * nr, V + size_t(k) * n, nullptr, h + size_t(k + 1) * nr);
      read_h(hh, k + 2);
      bool anyact = false;
      for (int c = 0; c < nr; ++c) {
        if (!act[c]) {
          denh[c] = 0.0;
          continue;
        }
        double* H = &Hs[size_t(c) * ldh * m];
        double* col = H + size_t(k) * ldh;
        for (int i = 0; i <= k; ++i) col[i] = hh[size_t(i) * nr + c];
        col[k + 1] = std::sqrt(hh[size_t(k + 1) * nr + c]);
        denh[c] = col[k + 1] > 0.0 ? col[k + 1] : 0.0;
        double* csc = &cs[size_t(c) * m];
        double* snc = &sn[size_t(c) * m];
        double* gc = &g[size_t(c) * ldh];
        for (int i = 0; i < k; ++i) {   // the earlier rotations on the new column
          const double t = csc[i] * col[i] + snc[i] * col[i + 1];
          col[i + 1] = -snc[i] * col[i] + csc[i] * col[i + 1];
          col[i] = t;
        }
        const double rho = std::hypot(col[k], col[k + 1]);
        if (!(rho > 0.0)) {   // breakdown without progress: end the cycle here
          act[c] = 0;
          denh[c] = 0.0;
          continue;
        }
        csc[k] = col[k] / rho;
        snc[k] = col[k + 1] / rho;
        col[k] = rho;
        col[k + 1] = 0.0;
        gc[k + 1] = -snc[k] * gc[k];
        gc[k] = csc[k] * gc[k];
        its[c] = it;
        kd[c] = k + 1;
        if (std::fabs(gc[k + 1]) <= tol * nf[c] || it >= maxit) {
          act[c] = 0;
          denh[c] = 0.0;
        }
        anyact = anyact || act[c];
      }
      if (!anyact) break;
      HIP_CHECK(hipMemcpyAsync(den, denh.data(), size_t(nr) * 8, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_gm_div, dim3(ne), dim3(kThreads), 0, st, n, nr, den, w,
                         V + size_t(k + 1) * n);
    }
    // y = R^-1 g (back substitution) per column, x += Z y
    int kmax = 0;
    std::fill(Yh.begin(), Yh.end(), 0.0);
    for (int c = 0; c < nr; ++c) {
      const int kc = kd[c];
      kmax = std::max(kmax, kc);
      const double* H = &Hs[size_t(c) * ldh * m];
      const double* gc = &g[size_t(c) * ldh];
      for (int i = kc - 1; i >= 0; --i) {
        double t = gc[i];
        for (int j = i + 1; j < kc; ++j) t -= H[i + size_t(j) * ldh] * Yh[size_t(j) * nr + c];
        Yh[size_t(i) * nr + c] = t / H[i + size_t(i) * ldh];
      }
      if (kc > 0 && std::fabs(gc[kc]) <= tol * nf[c]) live[c] = 0;
    }
    if (kmax > 0) {
      HIP_CHECK(hipMemcpyAsync(Yd, Yh.data(), size_t(kmax) * nr * 8, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL((k_gm_combine<TR>), dim3(ne), dim3(kThreads), 0, st, n, nr, kmax, Yd, Zk,
                         x);
    }
  }
  hipLaunchKernelGGL(k_to_colmajor<double>, dim3(ne), dim3(kThreads), 0, st, N, nr, x, u, ldu);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));
  bool converged = true;
  for (int c = 0; c < nr; ++c) {
    iters[c] = its[c];
    relres[c] = nf[c] > 0.0 ? std::sqrt(hh[c]) / nf[c] : 0.0;
    if (live[c]) converged = false;
  }
  return converged;
}

// Stencil assembly and the factorization of every level into F.
static void build_factor(hifde_factor_s& F, hifde_tree_s* tree, const double* const* a,
                         const double* b, double eps, hifde_precision prec, hipStream_t st) {
  F.g = tree->g;
  F.prec = prec;
  F.eps = eps;
  F.planner.reset(new Planner(F.g, tree->take_scratch()));
  F.cl.resize(F.g.L + 1);
  F.gl.resize(F.g.L);
  const int64_t N = F.g.N;
  F.diag.alloc(size_t(N) * 8);
  F.offd.alloc(size_t(N) * F.g.dim * 8);
  const double** aptr = F.mem.get<const double*>(F.g.dim);
  int* bad = F.mem.get<int>(1);
  std::vector<const double*> ah(a, a + F.g.dim);
  HIP_CHECK(hipMemcpyAsync(aptr, ah.data(), ah.size() * sizeof(void*), hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_stencil, dim3(nblk(N)), dim3(kThreads), 0, st, aptr, F.g.dim, F.g.n, N, b,
                     F.diag.as<double>(), F.offd.as<double>(), bad);
  HIP_CHECK(hipGetLastError());
  if (F.presize == 1) {
    F.offd_ev = F.new_event();
    HIP_CHECK(hipEventRecord(F.offd_ev, st));
  }
  // the flags are read at the first synchronization of the factorization
  // (check_input): until then every kernel indexes by structure only, so
  // invalid values cannot make one fault
  F.bad_d = bad;
  {
    // freed planners wait meanwhile (see planning_begin)
    struct Planning {
      Planning() { planning_begin(); }
      ~Planning() { planning_end(); }
    } planning;
    if (prec == HIFDE_MIXED) run_factor<float, float>(F, tree, st);
    else if (prec == HIFDE_MIXED_ELIM64) run_factor<double, float>(F, tree, st);
    else run_factor<double, double>(F, tree, st);
  }
  F.join_side(st);
  HIP_CHECK(hipStreamSynchronize(st));
  check_input(F, st);
  tree->give_scratch(F.planner->take_scratch());   // planning is over (not after a failure)
}

// Counts the bytes that differ between two device buffers.
__global__ void k_count_diff(int64_t n, const unsigned char* a, const unsigned char* b,
                             unsigned long long* cnt) {
  unsigned long long c = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    c += a[i] != b[i] ? 1ull : 0ull;
  if (c) atomicAdd(cnt, c);
}

// HIFDE_DEBUG_DETERMINISM: the skeleton choices and every stored value of
// two factorizations of the same input must agree bit for bit.
static void compare_factors(hifde_factor_s& A, hifde_factor_s& B, hipStream_t st) {
  DevMem cnt;
  cnt.alloc(8);
  unsigned long long* c = cnt.as<unsigned long long>();
  auto same = [&](const void* x, const void* y, size_t bytes, const char* what, int l) {
    if (bytes == 0) return;
    HIP_CHECK(hipMemsetAsync(c, 0, 8, st));
    hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(kThreads), 0, st, int64_t(bytes),
                       static_cast<const unsigned char*>(x), static_cast<const unsigned char*>(y), c);
    unsigned long long h = 0;
    HIP_CHECK(hipMemcpyAsync(&h, c, 8, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    if (h) {
      char buf[160];
      snprintf(buf, sizeof buf, "nondeterministic factorization: %llu bytes of %s differ at level %d",
               h, what, l);
      throw Error(HIFDE_EDEVICE, buf);
    }
  };
  const int L = A.g.L;
  for (int l = 0; l <= L; ++l) {
    const size_t esz = (l == L || !float_sweeps(A)) ? 8 : 4;
    const SweepSet& S = A.cl[l].st->sw;
    same(A.cl[l].pk, B.cl[l].pk, size_t(S.pk_elems) * esz, "cell factors", l);
    same(A.cl[l].dinv, B.cl[l].dinv, size_t(S.dv_elems) * esz, "cell pivots", l);
    if (l == L) continue;
    const GroupLevel& GA = A.gl[l];
    const GroupLevel& GB = B.gl[l];
    if (GA.nskel != GB.nskel || GA.gsel_h != GB.gsel_h || GA.idx_h != GB.idx_h)
      throw Error(HIFDE_EDEVICE, "nondeterministic skeleton choice at level " + std::to_string(l));
    same(GA.pk, GB.pk, size_t(GA.sw.pk_elems) * esz, "skeleton-front factors", l);
    same(GA.tpool, GB.tpool, size_t(GA.st->t_elems) * esz, "interpolation matrices", l);
  }
}


}  // namespace hifde

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* hifde_last_error(void) { return g_last_error.c_str(); }

int hifde_build_tree(int dim, int64_t n, int64_t leaf, int skip_levels, hifde_tree_t* out) {
  if (!out) return fail(HIFDE_EINVAL, "out is NULL");
  *out = nullptr;
  Geom g;
  std::string err = check_geom(dim, n, leaf, skip_levels, &g);
  if (!err.empty()) return fail(HIFDE_EINVAL, err);
  return guarded([&] {
    auto* t = new hifde_tree_s;
    t->g = g;
    *out = t;
  });
}

void hifde_tree_free(hifde_tree_t tree) { delete tree; }

int hifde_tree_set_memory_limit(hifde_tree_t tree, int64_t bytes) {
  if (!tree) return fail(HIFDE_EINVAL, "NULL tree");
  if (bytes < 0) return fail(HIFDE_EINVAL, "bytes must be >= 0");
  tree->pool->limit = size_t(bytes);
  return HIFDE_OK;
}

void hifde_factor_free(hifde_factor_t F) {
  if (!F) return;
  PhaseTimer tm;
  F->release_handles();
  tm.mark("free: handles", -1);
  F->cl.clear();
  F->gl.clear();
  tm.mark("free: levels", -1);
  discard_planner(std::move(F->planner));
  tm.mark("free: planner", -1);
  delete F;
  tm.mark("free: rest", -1);
}

int hifde_factor(hifde_tree_t tree, const double* const* a, const double* b, double eps,
                 hifde_precision prec, uint32_t flags, void* hip_stream, hifde_factor_t* out) {
  if (!out) return fail(HIFDE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!tree || !a) return fail(HIFDE_EINVAL, "tree or a is NULL");
  if (!(eps >= 0.0 && eps < 1.0)) return fail(HIFDE_EINVAL, "eps must lie in [0, 1)");
  if (prec != HIFDE_FP64 && prec != HIFDE_MIXED && prec != HIFDE_MIXED_ELIM64)
    return fail(HIFDE_EINVAL, "unknown precision");
  if (flags & ~uint32_t(HIFDE_USE_RANK_MODEL | HIFDE_DEBUG_DETERMINISM | HIFDE_AUTOTUNE |
                        HIFDE_NO_GRAPH | HIFDE_PRESIZE_WORST_CASE | HIFDE_SWEEP_ROW_TILES |
                        HIFDE_INDEFINITE | HIFDE_SKETCH_ID | HIFDE_RETRY_FP64))
    return fail(HIFDE_EINVAL, "unknown flags");
  if ((flags & HIFDE_USE_RANK_MODEL) && (flags & HIFDE_PRESIZE_WORST_CASE))
    return fail(HIFDE_EINVAL, "HIFDE_USE_RANK_MODEL and HIFDE_PRESIZE_WORST_CASE exclude each other");
  if ((flags & HIFDE_USE_RANK_MODEL) && tree && tree->model.empty())
    return fail(HIFDE_ESTATE, "HIFDE_USE_RANK_MODEL without a rank model on the tree");
  for (int k = 0; k < tree->g.dim; ++k)
    if (!a[k]) return fail(HIFDE_EINVAL, "a[k] is NULL");
  std::unique_ptr<hifde_factor_s> F(new hifde_factor_s);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int rc = guarded([&] {
    auto t0 = std::chrono::steady_clock::now();
    const int presize = (flags & HIFDE_USE_RANK_MODEL) ? 1 : (flags & HIFDE_PRESIZE_WORST_CASE) ? 2 : 0;
    auto setup = [&](hifde_factor_s& G) {
      G.presize = presize;
      G.model = presize == 1 ? tree->model_d.as<float>() : nullptr;
      G.autotune = (flags & HIFDE_AUTOTUNE) != 0;
      G.definite = !(flags & HIFDE_INDEFINITE);
      G.sketch = (flags & HIFDE_SKETCH_ID) != 0;
      G.tree = tree;
      G.use_pool(tree->pool);
    };
    setup(*F);
    bool retried = false;
    try {
      build_factor(*F, tree, a, b, eps, prec, st);
    } catch (const Error& e) {
      // a pivot of the float factorization failed: factor again in double
      if (!(flags & HIFDE_RETRY_FP64) || e.code != HIFDE_ENOTSPD || prec == HIFDE_FP64) throw;
      HIP_CHECK(hipStreamSynchronize(st));
      F.reset(new hifde_factor_s);
      setup(*F);
      prec = HIFDE_FP64;
      retried = true;
      build_factor(*F, tree, a, b, eps, prec, st);
    }
    F->use_graph = !(flags & HIFDE_NO_GRAPH);
    F->row_tiles = (flags & HIFDE_SWEEP_ROW_TILES) != 0;
    fill_stats(*F);
    F->stats.retried = retried ? 1 : 0;
    F->stats.factor_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (flags & HIFDE_DEBUG_DETERMINISM) {
      hifde_factor_s F2;
      F2.use_pool(tree->pool);
      F2.presize = presize;
      F2.model = F->model;
      F2.definite = F->definite;
      F2.sketch = F->sketch;
      F2.tree = tree;
      build_factor(F2, tree, a, b, eps, prec, st);
      compare_factors(*F, F2, st);
    }
  });
  if (rc == HIFDE_OK) *out = F.release();
  return rc;
}

int hifde_plan_replay(hifde_tree_t tree, const int32_t* redundant_level, hifde_factor_t* out) {
  if (!out) return fail(HIFDE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!tree || !redundant_level) return fail(HIFDE_EINVAL, "tree or redundant_level is NULL");
  std::unique_ptr<hifde_factor_s> F(new hifde_factor_s);
  int rc = guarded([&] {
    F->g = tree->g;
    F->plan_only = true;
    F->planner.reset(new Planner(F->g));
    Planner& P = *F->planner;
    PhaseTimer tm;
    for (int l = 0; l < F->g.L; ++l) {
      P.plan_cells(l);
      tm.mark("plan cells", l);
      P.plan_groups(l);
      tm.mark("plan groups", l);
      const auto& groups = P.level(l).groups();
      size_t stride = 1;
      for (const auto& G : groups) stride = std::max(stride, G.c.size());
      std::vector<int32_t> ks(groups.size()), pos(groups.size() * stride);
      for (size_t gi = 0; gi < groups.size(); ++gi) {
        // skeleton positions listed in decreasing order (set_skeletons sorts)
        int k = 0;
        for (int32_t i = int32_t(groups[gi].c.size()) - 1; i >= 0; --i)
          if (redundant_level[groups[gi].c[i]] != 2 * l + 1) pos[gi * stride + size_t(k++)] = i;
        ks[gi] = k;
      }
      tm.mark("skeleton positions", l);
      P.set_skeletons(l, ks.data(), pos.data(), stride);
      tm.mark("set skeletons", l);
      P.finish_groups(l);
      tm.mark("finish groups", l);
    }
    P.plan_cells(F->g.L);
    F->prec = HIFDE_FP64;
    fill_stats(*F);
  });
  if (rc == HIFDE_OK) *out = F.release();
  return rc;
}

int hifde_stats(hifde_factor_t F, hifde_stats_t* out) {
  if (!F || !out) return fail(HIFDE_EINVAL, "NULL argument");
  *out = F->stats;
  return HIFDE_OK;
}

int hifde_profile(hifde_factor_t F, uint32_t class_mask, int level) {
  if (!F) return fail(HIFDE_EINVAL, "NULL factor");
  if (class_mask >> HIFDE_PROF_CLASSES) return fail(HIFDE_EINVAL, "unknown kernel class");
  if (level < -1 || level > F->g.L) return fail(HIFDE_EINVAL, "level out of range");
  F->prof_mask = class_mask;
  F->prof_level = level;
  return HIFDE_OK;
}

int hifde_profile_read(hifde_factor_t F, int cls, hifde_prof_t* out) {
  if (!F || !out) return fail(HIFDE_EINVAL, "NULL argument");
  if (cls < 0 || cls >= HIFDE_PROF_CLASSES) return fail(HIFDE_EINVAL, "unknown kernel class");
  return guarded([&] {
    prof_collect(*F);
    *out = F->prof_acc[cls];
    F->prof_acc[cls] = hifde_prof_t{};
  });
}

int hifde_mlp_workspace(int64_t nbatch, int64_t* bytes) {
  if (!bytes || nbatch < 1) return fail(HIFDE_EINVAL, "bad arguments");
  *bytes = (int64_t(4) * kRankH + 2) * 4 * nbatch;
  return HIFDE_OK;
}

int hifde_mlp_forward(const float* params, int64_t nbatch, const float* feat, float* out,
                      void* hip_stream) {
  if (!params || !feat || !out || nbatch < 1) return fail(HIFDE_EINVAL, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return guarded([&] {
    hipLaunchKernelGGL(k_mlp_forward, dim3(nblk(nbatch)), dim3(kThreads), 0, st, params, nbatch,
                       feat, out, static_cast<float*>(nullptr), static_cast<float*>(nullptr));
    HIP_CHECK(hipGetLastError());
  });
}

// The four launches of one gradient: forward with the activations kept,
// backward through them, the parameter gradient and the loss.  work holds
// y, dy (nbatch each) and h1, h2, dz1, dz2 (nbatch x kRankH each); every
// launch writes its part of it for all nbatch samples before any reads it.
static void mlp_grad_launch(const float* params, int64_t nbatch, const float* feat,
                            const float* target, float* grad, float* loss, float* work,
                            hipStream_t st) {
  float* y = work;
  float* dy = y + nbatch;
  float* h1 = dy + nbatch;
  float* h2 = h1 + nbatch * kRankH;
  float* dz1 = h2 + nbatch * kRankH;
  float* dz2 = dz1 + nbatch * kRankH;
  hipLaunchKernelGGL(k_mlp_forward, dim3(nblk(nbatch)), dim3(kThreads), 0, st, params, nbatch,
                     feat, y, h1, h2);
  hipLaunchKernelGGL(k_mlp_backprop, dim3(nblk(nbatch)), dim3(kThreads), 0, st, params, nbatch,
                     y, target, h1, h2, dy, dz1, dz2);
  hipLaunchKernelGGL(k_mlp_param_grad, dim3(nblk(kRankP)), dim3(kThreads), 0, st, nbatch, feat,
                     h1, h2, dy, dz1, dz2, grad);
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(kThreads), 0, st, nbatch, y, target, loss);
  HIP_CHECK(hipGetLastError());
}

int hifde_mlp_grad(const float* params, int64_t nbatch, const float* feat, const float* target,
                   float* grad, float* loss, void* work, void* hip_stream) {
  if (!params || !feat || !target || !grad || !loss || !work || nbatch < 1)
    return fail(HIFDE_EINVAL, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return guarded([&] {
    mlp_grad_launch(params, nbatch, feat, target, grad, loss, static_cast<float*>(work), st);
  });
}

// Workspace of hifde_mlp_grad_noalloc: the activations and their gradients
// of up to HIFDE_MLP_NOALLOC_MAX_BATCH samples.  Each device holds its own
// copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns on that device (the array's name in
// host code is not a device address).
constexpr int64_t kMlpStaticBatch = HIFDE_MLP_NOALLOC_MAX_BATCH;
static __device__ __align__(256) float mlp_scratch[(4 * kRankH + 2) * kMlpStaticBatch];

constexpr int kMaxDevices = 64;
static std::mutex g_mlp_scratch_mu;
static float* g_mlp_scratch[kMaxDevices] = {};

// Device address of mlp_scratch on the current device, looked up on the
// first call on that device and kept.
static float* mlp_scratch_address() {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(HIFDE_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mlp_scratch_mu);
  if (!g_mlp_scratch[dev]) {
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(mlp_scratch)));
    if (!p) throw Error(HIFDE_EDEVICE, "no device address for the static workspace");
    g_mlp_scratch[dev] = static_cast<float*>(p);
  }
  return g_mlp_scratch[dev];
}

int hifde_mlp_grad_noalloc(const float* params, int64_t nbatch, const float* feat,
                           const float* target, float* grad, float* loss, void* hip_stream) {
  if (!params || !feat || !target || !grad || !loss || nbatch < 1)
    return fail(HIFDE_EINVAL, "bad arguments");
  if (nbatch > kMlpStaticBatch)
    return fail(HIFDE_EINVAL, "nbatch exceeds HIFDE_MLP_NOALLOC_MAX_BATCH");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return guarded([&] {
    mlp_grad_launch(params, nbatch, feat, target, grad, loss, mlp_scratch_address(), st);
  });
}

int hifde_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr,
                   void* hip_stream) {
  if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0f))
    return fail(HIFDE_EINVAL, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return guarded([&] {
    hipLaunchKernelGGL(k_mlp_adam, dim3(nblk(kRankP)), dim3(kThreads), 0, st, params, grad, m, v,
                       step, lr, 0.9f, 0.999f, 1e-8f);
    HIP_CHECK(hipGetLastError());
  });
}

int hifde_rank_features(hifde_factor_t F, int level, float* feat, float* target, int64_t cap,
                        int64_t* ngroups, void* hip_stream) {
  if (!F || !ngroups) return fail(HIFDE_EINVAL, "NULL argument");
  if (F->plan_only) return fail(HIFDE_ESTATE, "factor holds no numerical data");
  if (level < 0 || level >= F->g.L) return fail(HIFDE_EINVAL, "level out of range");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return guarded([&] {
    const Level& lev = F->planner->level(level);
    const int64_t ng = int64_t(lev.groups().size());
    *ngroups = ng;
    if (!feat) return;
    if (cap < ng) throw Error(HIFDE_EINVAL, "cap is smaller than the number of groups");
    group_features(*F, level, feat, st);
    if (target) {
      std::vector<float> t(ng);
      for (int64_t g = 0; g < ng; ++g) t[g] = float(std::log2(1.0 + double(lev.res[g].k)));
      HIP_CHECK(hipMemcpyAsync(target, t.data(), ng * 4, hipMemcpyHostToDevice, st));
      HIP_CHECK(hipStreamSynchronize(st));
    }
  });
}

int hifde_set_rank_model(hifde_tree_t tree, const float* weights, int64_t nweights) {
  if (!tree) return fail(HIFDE_EINVAL, "NULL tree");
  if (weights && nweights != kRankP) return fail(HIFDE_EINVAL, "nweights must be HIFDE_RANK_PARAMS");
  return guarded([&] {
    if (!weights) {
      tree->model.clear();
      tree->model_d.release();
      return;
    }
    tree->model.assign(weights, weights + nweights);
    tree->model_d.alloc(size_t(kRankP) * 4);
    HIP_CHECK(hipMemcpy(tree->model_d.p, weights, size_t(kRankP) * 4, hipMemcpyHostToDevice));
  });
}

int hifde_export_sets(hifde_factor_t F, int level2, hifde_sets_t* out) {
  if (!F || !out) return fail(HIFDE_EINVAL, "NULL argument");
  const int L = F->g.L;
  if (level2 < 0 || level2 > 2 * L) return fail(HIFDE_EINVAL, "level2 out of range");
  return guarded([&] {
    const Level& lev = F->planner->level(level2 / 2);
    std::vector<int64_t> ids;
    std::vector<const std::vector<int32_t>*> lists[4];
    std::vector<int32_t> empty;
    if (level2 % 2 == 0) {
      for (const Cell& c : lev.cells()) {
        ids.push_back(c.cid);
        lists[0].push_back(&c.p);
        lists[1].push_back(&c.q);
        lists[2].push_back(&empty);
        lists[3].push_back(&empty);
      }
    } else {
      for (size_t gi = 0; gi < lev.groups().size(); ++gi) {
        const Group& g = lev.groups()[gi];
        const GroupRes& R = lev.res[gi];
        ids.push_back(g.gid);
        lists[0].push_back(&g.c);
        lists[1].push_back(&g.cN);
        lists[2].push_back(R.skel ? &R.sk : &g.c);
        lists[3].push_back(R.skel ? &R.rd : &empty);
      }
    }
    out->count = int64_t(ids.size());
    for (int w = 0; w < 4; ++w) {
      int64_t tot = 0;
      for (auto* v : lists[w]) tot += int64_t(v->size());
      out->total[w] = tot;
    }
    if (out->ids) std::copy(ids.begin(), ids.end(), out->ids);
    for (int w = 0; w < 4; ++w) {
      if (!out->offs[w] && !out->lists[w]) continue;
      int64_t o = 0;
      for (size_t i = 0; i < lists[w].size(); ++i) {
        if (out->offs[w]) out->offs[w][i] = o;
        if (out->lists[w]) std::copy(lists[w][i]->begin(), lists[w][i]->end(), out->lists[w] + o);
        o += int64_t(lists[w][i]->size());
      }
      if (out->offs[w]) out->offs[w][lists[w].size()] = o;
    }
  });
}

int hifde_solve(hifde_factor_t F, int64_t nrhs, const double* f, int64_t ldf, double* u,
                int64_t ldu, void* hip_stream) {
  if (!F || !f || !u) return fail(HIFDE_EINVAL, "NULL argument");
  if (F->plan_only) return fail(HIFDE_ESTATE, "factor holds no numerical data");
  if (nrhs < 1 || ldf < F->g.N || ldu < F->g.N) return fail(HIFDE_EINVAL, "bad nrhs or ld");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return guarded([&] {
    const int64_t N = F->g.N, n = N * nrhs;
    ensure_X(*F, nrhs);
    if (float_sweeps(*F)) {
      float* X = F->X.as<float>();
      hipLaunchKernelGGL(k_from_colmajor<float>, dim3(nblk(n)), dim3(kThreads), 0, st, N, int(nrhs),
                         f, ldf, X);
      apply_inverse_g<float, float>(*F, X, F->Z.as<float>(), int(nrhs), st);
      hipLaunchKernelGGL(k_to_colmajor<float>, dim3(nblk(n)), dim3(kThreads), 0, st, N, int(nrhs),
                         X, u, ldu);
    } else {
      double* X = F->X.as<double>();
      hipLaunchKernelGGL(k_from_colmajor<double>, dim3(nblk(n)), dim3(kThreads), 0, st, N,
                         int(nrhs), f, ldf, X);
      apply_inverse_g<double, double>(*F, X, F->Z.as<double>(), int(nrhs), st);
      hipLaunchKernelGGL(k_to_colmajor<double>, dim3(nblk(n)), dim3(kThreads), 0, st, N,
                         int(nrhs), X, u, ldu);
    }
    HIP_CHECK(hipGetLastError());
  });
}

int hifde_matvec(hifde_factor_t F, int64_t nrhs, const double* x, int64_t ldx, double* y,
                 int64_t ldy, void* hip_stream) {
  if (!F || !x || !y) return fail(HIFDE_EINVAL, "NULL argument");
  if (F->plan_only) return fail(HIFDE_ESTATE, "factor holds no numerical data");
  if (nrhs < 1 || ldx < F->g.N || ldy < F->g.N) return fail(HIFDE_EINVAL, "bad nrhs or ld");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return guarded([&] {
    const int64_t N = F->g.N, n = N * nrhs;
    DevMem a, b;
    a.alloc(size_t(n) * 8);
    b.alloc(size_t(n) * 8);
    hipLaunchKernelGGL(k_from_colmajor<double>, dim3(nblk(n)), dim3(kThreads), 0, st, N, int(nrhs),
                       x, ldx, a.as<double>());
    hipLaunchKernelGGL(k_matvec, dim3(nblk(n)), dim3(kThreads), 0, st, N, int(nrhs), F->g.dim,
                       F->g.n, F->diag.as<double>(), F->offd.as<double>(), a.as<double>(),
                       b.as<double>());
    hipLaunchKernelGGL(k_to_colmajor<double>, dim3(nblk(n)), dim3(kThreads), 0, st, N, int(nrhs),
                       b.as<double>(), y, ldy);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
  });
}

int hifde_pcg(hifde_factor_t F, int64_t nrhs, const double* f, int64_t ldf, double* u, int64_t ldu,
              double tol, int maxit, int* iters, double* relres, void* hip_stream) {
  if (!F || !f || !u || !iters || !relres) return fail(HIFDE_EINVAL, "NULL argument");
  if (F->plan_only) return fail(HIFDE_ESTATE, "factor holds no numerical data");
  if (nrhs < 1 || ldf < F->g.N || ldu < F->g.N) return fail(HIFDE_EINVAL, "bad nrhs or ld");
  if (!(tol > 0.0) || maxit < 1) return fail(HIFDE_EINVAL, "tol must be > 0 and maxit >= 1");
  if (!F->definite)
    return fail(HIFDE_ESTATE, "the factor is indefinite (HIFDE_INDEFINITE): use hifde_gmres");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  bool converged = true;
  int rc = guarded([&] {
    if (float_sweeps(*F))
      converged = run_pcg<float>(*F, nrhs, f, ldf, u, ldu, tol, maxit, iters, relres, st);
    else
      converged = run_pcg<double>(*F, nrhs, f, ldf, u, ldu, tol, maxit, iters, relres, st);
  });
  if (rc != HIFDE_OK) return rc;
  if (!converged) return fail(HIFDE_ENOCONV, "PCG did not reach the tolerance within maxit");
  return HIFDE_OK;
}

int hifde_gmres(hifde_factor_t F, int64_t nrhs, const double* f, int64_t ldf, double* u,
                int64_t ldu, double tol, int restart, int maxit, int* iters, double* relres,
                void* hip_stream) {
  if (!F || !f || !u || !iters || !relres) return fail(HIFDE_EINVAL, "NULL argument");
  if (F->plan_only) return fail(HIFDE_ESTATE, "factor holds no numerical data");
  if (nrhs < 1 || ldf < F->g.N || ldu < F->g.N) return fail(HIFDE_EINVAL, "bad nrhs or ld");
  if (!(tol > 0.0 && tol < HUGE_VAL) || maxit < 1 || restart < 1)
    return fail(HIFDE_EINVAL, "tol must be finite and > 0, maxit and restart >= 1");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  bool converged = true;
  int rc = guarded([&] {
    if (float_sweeps(*F))
      converged =
          run_gmres<float>(*F, nrhs, f, ldf, u, ldu, tol, restart, maxit, iters, relres, st);
    else
      converged =
          run_gmres<double>(*F, nrhs, f, ldf, u, ldu, tol, restart, maxit, iters, relres, st);
  });
  if (rc != HIFDE_OK) return rc;
  if (!converged) return fail(HIFDE_ENOCONV, "GMRES did not reach the tolerance within maxit");
  return HIFDE_OK;
}

}  // extern "C"
