// Host-side tree and per-level plans of HIF-DE; see planner.hpp.
#include "planner.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <condition_variable>
#include <cstdlib>
#include <exception>
#include <functional>
#include <mutex>
#include <stdexcept>
#include <thread>

namespace hifde {

// A process-wide pool of planning threads: started once, parked on a
// condition variable between jobs.  A job is a function of (item, worker)
// over [0, n), taken `grain` items at a time from an atomic counter; the
// calling thread works as worker 0.  One job runs at a time.
namespace {
// Spins briefly (a waiting thread is usually needed again within a few tens
// of microseconds while a level is planned) before blocking.
inline void cpu_relax() {
#if defined(__x86_64__)
  __builtin_ia32_pause();
#else
  std::this_thread::yield();
#endif
}
constexpr auto kSpin = std::chrono::microseconds(200);

class PlanPool {
 public:
  static PlanPool& get() {
    static PlanPool pool;
    return pool;
  }
  int size() const { return int(threads_.size()) + 1; }

  void run(size_t n, size_t grain, int workers, const std::function<void(size_t, int)>& f) {
    std::lock_guard<std::mutex> one(job_mutex_);
    const int helpers = std::min<int>(workers, size()) - 1;
    {
      std::lock_guard<std::mutex> lk(m_);
      fn_ = &f;
      n_ = n;
      grain_ = grain;
      next_.store(0);
      failed_.store(false);
      err_ = nullptr;
      helpers_ = helpers;
      pending_.store(helpers);
      epoch_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    work(0);
    const auto t0 = std::chrono::steady_clock::now();
    while (pending_.load(std::memory_order_acquire) != 0 &&
           std::chrono::steady_clock::now() - t0 < kSpin)
      cpu_relax();
    std::unique_lock<std::mutex> lk(m_);
    done_.wait(lk, [&] { return pending_.load() == 0; });
    fn_ = nullptr;
    if (err_) std::rethrow_exception(err_);
  }

 private:
  PlanPool() {
    // two CPUs left to the factorization's other host threads (the
    // skeleton-front helper, the HIP runtime's): a pool that fills every
    // CPU stalls on them
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int n = std::max(1, int(std::min(16u, hw)) - 2);
    if (const char* e = std::getenv("HIFDE_PLAN_THREADS")) n = std::max(1, std::atoi(e));
    for (int w = 1; w < n; ++w) threads_.emplace_back([this, w] { loop(w); });
  }
  ~PlanPool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_.store(true);
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }
  void work(int w) {
    try {
      for (;;) {
        const size_t b = next_.fetch_add(grain_);
        if (b >= n_ || failed_.load()) break;
        const size_t e = std::min(n_, b + grain_);
        for (size_t i = b; i < e; ++i) (*fn_)(i, w);
      }
    } catch (...) {
      std::lock_guard<std::mutex> lk(m_);
      if (!failed_.exchange(true)) err_ = std::current_exception();
    }
  }
  void loop(int w) {
    uint64_t seen = 0;
    for (;;) {
      const auto t0 = std::chrono::steady_clock::now();
      while (epoch_.load(std::memory_order_acquire) == seen && !stop_.load() &&
             std::chrono::steady_clock::now() - t0 < kSpin)
        cpu_relax();
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return stop_.load() || epoch_.load() != seen; });
        if (stop_.load()) return;
        seen = epoch_.load();
        if (w > helpers_) continue;   // not needed for this job
      }
      work(w);
      if (pending_.fetch_sub(1, std::memory_order_acq_rel) == 1) {
        std::lock_guard<std::mutex> lk(m_);
        done_.notify_one();
      }
    }
  }

  std::vector<std::thread> threads_;
  std::mutex m_, job_mutex_;
  std::condition_variable cv_, done_;
  const std::function<void(size_t, int)>* fn_ = nullptr;
  size_t n_ = 0, grain_ = 1;
  std::atomic<size_t> next_{0};
  std::atomic<bool> failed_{false};
  std::exception_ptr err_;
  int helpers_ = 0;
  std::atomic<int> pending_{0};
  std::atomic<uint64_t> epoch_{0};
  std::atomic<bool> stop_{false};
};

// Frees finished planners on a background thread: their level plans are
// many small host arrays, whose release would otherwise hold up the caller.
// It waits while a factorization is planning (planning_begin/end): freeing
// beside the planner's threads slowed their allocations.
class Janitor {
 public:
  static Janitor& get() {
    static Janitor j;
    return j;
  }
  void discard(std::unique_ptr<Planner> p) {
    {
      std::lock_guard<std::mutex> lk(m_);
      q_.push_back(std::move(p));
    }
    cv_.notify_one();
  }
  void planning(int delta) {
    {
      std::lock_guard<std::mutex> lk(m_);
      active_ += delta;
    }
    cv_.notify_one();
  }

 private:
  Janitor() : t_([this] { loop(); }) {}
  ~Janitor() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
    }
    cv_.notify_one();
    t_.join();
  }
  void loop() {
    std::unique_lock<std::mutex> lk(m_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || (!q_.empty() && active_ == 0); });
      if (stop_ && (q_.empty() || active_ > 0)) return;   // stopping
      std::vector<std::unique_ptr<Planner>> batch;
      batch.swap(q_);
      lk.unlock();
      batch.clear();
      lk.lock();
    }
  }
  std::mutex m_;
  std::condition_variable cv_;
  std::vector<std::unique_ptr<Planner>> q_;
  int active_ = 0;   // factorizations planning
  bool stop_ = false;
  std::thread t_;   // last: starts once the members above exist
};
}  // namespace

// Section times of one planning step, printed under HIFDE_TIMING.
struct PlanTimer {
  bool on = std::getenv("HIFDE_TIMING") != nullptr;
  int level;
  const char* step;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  PlanTimer(const char* s, int l) : level(l), step(s) {}
  void mark(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[hifde] level %d     %s: %-16s %8.3f ms\n", level, step, what,
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

// Runs f(i, worker) for i in [0, n) on up to `workers` threads (worker ids
// below `workers`), `grain` items at a time; the first exception is
// rethrown here.
template <class F>
static void parallel_for(size_t n, size_t grain, int workers, F&& f) {
  const size_t chunks = (n + grain - 1) / grain;
  const int nt = int(std::min<size_t>(size_t(workers), chunks));
  if (nt <= 1) {
    for (size_t i = 0; i < n; ++i) f(i, 0);
    return;
  }
  const std::function<void(size_t, int)> fn = [&](size_t i, int w) { f(i, w); };
  PlanPool::get().run(n, grain, nt, fn);
}

// Stable grouping of the items i with key[i] >= 0 by key (a counting sort
// over contiguous blocks of items, so the order inside a key is the items'
// order): start[k] .. start[k+1] - 1 index `order` for key k.
static void bucket_by_key(const std::vector<int32_t>& key, int64_t nkey, int workers,
                          std::vector<int32_t>& start, std::vector<int32_t>& order) {
  const size_t n = key.size();
  const size_t nb = std::max<size_t>(1, std::min<size_t>(64, (n + 4095) / 4096));
  std::vector<int32_t> hist(nb * size_t(nkey), 0);
  auto range = [&](size_t b, size_t* lo, size_t* hi) {
    *lo = n * b / nb;
    *hi = n * (b + 1) / nb;
  };
  parallel_for(nb, 1, workers, [&](size_t b, int) {
    size_t lo, hi;
    range(b, &lo, &hi);
    int32_t* h = hist.data() + b * size_t(nkey);
    for (size_t i = lo; i < hi; ++i)
      if (key[i] >= 0) ++h[key[i]];
  });
  start.assign(size_t(nkey) + 1, 0);
  for (int64_t k = 0; k < nkey; ++k) {
    int32_t run = start[k];
    for (size_t b = 0; b < nb; ++b) {
      const int32_t c = hist[b * size_t(nkey) + k];
      hist[b * size_t(nkey) + k] = run;   // this block's first slot for key k
      run += c;
    }
    start[k + 1] = run;
  }
  order.resize(size_t(start[nkey]));
  parallel_for(nb, 1, workers, [&](size_t b, int) {
    size_t lo, hi;
    range(b, &lo, &hi);
    int32_t* h = hist.data() + b * size_t(nkey);
    for (size_t i = lo; i < hi; ++i)
      if (key[i] >= 0) order[h[key[i]]++] = int32_t(i);
  });
}

std::string check_geom(int dim, int64_t n, int64_t leaf, int skip, Geom* out) {
  if (dim != 2 && dim != 3) return "dim must be 2 or 3";
  if (leaf < 2) return "leaf must be at least 2";
  if (n <= leaf) return "n must hold at least two leaf boxes per side";
  // ceil(n/leaf) leaf boxes per side, the last one possibly short: a power
  // of two, so that every box of every level keeps unknowns to eliminate
  const int64_t B = (n + leaf - 1) / leaf;
  if ((B & (B - 1)) != 0) return "ceil(n/leaf) must be a power of two";
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

Planner::Planner(const Geom& g, std::unique_ptr<PlanScratch> scratch) : g_(g) {
  if (scratch) {
    loc_ = std::move(scratch->loc);
    own0_ = std::move(scratch->own0);
    own1_ = std::move(scratch->own1);
    act_ = std::move(scratch->act);
    act_spare_ = std::move(scratch->act_spare);
    active_ = std::move(scratch->active);
    grouped_ = std::move(scratch->grouped);
    geo_ = std::move(scratch->geo);
    active0_ = std::move(scratch->active0);
    act0_ = std::move(scratch->act0);
  }
  active_.assign(g_.N, 1);
  grouped_.assign(g_.N, 0);
  workers_ = PlanPool::get().size();
  loc_.resize(workers_);
  for (auto& v : loc_)
    if (!v.empty() && int64_t(v.size()) != g_.N) v.clear();   // re-made on first use
  if (int64_t(own0_.size()) != g_.N) own0_.assign(g_.N, -1);
  if (int64_t(own1_.size()) != g_.N) own1_.assign(g_.N, -1);
  act_.clear();   // every unknown: filled by the first plan_cells(0) or adopt_level0
  lv_.resize(g_.L + 1);
  // x lies on a level-l separator iff (x+1) mod (m 2^l) == 0 and x != n-1;
  // these sets are nested, so one number per coordinate describes them.
  seplev_.assign(g_.n, -1);
  for (int64_t x = 0; x < g_.n; ++x)
    for (int l = 0; l < g_.L; ++l) {
      const int64_t M = g_.m << l;
      if ((x + 1) % M == 0 && x != g_.n - 1) seplev_[x] = int8_t(l);
    }
  if (int64_t(geo_.size()) != g_.N) {
    geo_.resize(g_.N);
    parallel_for(size_t(g_.N), 65536, workers_, [&](size_t d, int) {
      int64_t x[3];
      coords(int64_t(d), x);
      uint32_t v = 0x00FFFFFFu;
      for (int k = 0; k < g_.dim; ++k) {
        v &= ~(0xFFu << (8 * k));
        v |= uint32_t(uint8_t(seplev_[x[k]])) << (8 * k);
        if (x[k] > 0) v |= 1u << (24 + 2 * k);
        if (x[k] < g_.n - 1) v |= 2u << (24 + 2 * k);
      }
      geo_[d] = v;
    });
  }
}

std::unique_ptr<PlanScratch> Planner::take_scratch() {
  auto s = std::make_unique<PlanScratch>();
  s->loc = std::move(loc_);
  s->own0 = std::move(own0_);
  s->own1 = std::move(own1_);
  s->act = std::move(act_);
  s->act_spare = std::move(act_spare_);
  s->active = std::move(active_);
  s->grouped = std::move(grouped_);
  s->geo = std::move(geo_);
  s->active0 = std::move(active0_);
  s->act0 = std::move(act0_);
  geo_.clear();
  active0_.clear();
  act0_.clear();
  loc_.clear();
  own0_.clear();
  own1_.clear();
  act_.clear();
  act_spare_.clear();
  active_.clear();
  grouped_.clear();
  return s;
}

void Planner::coords(int64_t d, int64_t* x) const {
  x[0] = d % g_.n;
  if (g_.dim > 1) x[1] = (d / g_.n) % g_.n;
  if (g_.dim > 2) x[2] = d / (g_.n * g_.n);
}

int Planner::sigma(int64_t d, int l) const {
  const uint32_t v = geo_[d];
  return int(int8_t(v) >= l) + int(int8_t(v >> 8) >= l) + int(int8_t(v >> 16) >= l);
}

int64_t Planner::box_of(int64_t d, int l) const {
  if (l >= g_.L) return 0;
  int64_t x[3];
  coords(d, x);
  const int64_t M = g_.m << l, B = (g_.n + M - 1) / M;
  int64_t id = 0, mul = 1;
  for (int k = 0; k < g_.dim; ++k) {
    id += (x[k] / M) * mul;
    mul *= B;
  }
  return id;
}

// k * B^dim + lexicographic(box indices), with the separator axis k.
int64_t Planner::group_key(int64_t d, int l) const {
  int64_t x[3];
  coords(d, x);
  const int64_t M = g_.m << l, B = (g_.n + M - 1) / M;
  int64_t id = 0, mul = 1;
  int axis = 0;
  for (int k = 0; k < g_.dim; ++k) {
    if (seplev_[x[k]] >= l) axis = k;
    id += (x[k] / M) * mul;
    mul *= B;
  }
  return int64_t(axis) * mul + id;
}

template <class F>
void Planner::for_neighbors(int64_t d, F&& f) const {
  const uint32_t b = geo_[d] >> 24;
  for (int k = 0; k < g_.dim; ++k) {
    if (b & (1u << (2 * k))) f(d - g_.stride[k], k, /*up=*/false);
    if (b & (2u << (2 * k))) f(d + g_.stride[k], k, /*up=*/true);
  }
}

static inline int64_t link_ref(int64_t N, int64_t lo, int k) { return N * (1 + k) + lo; }

// Start of every per-item map list in the concatenation of `parts`
// (reported through shift(i, start)); returns the total length.
template <class Shift>
static int64_t concat_offsets(const std::vector<std::vector<int32_t>>& parts, Shift&& shift) {
  int64_t base = 0;
  for (size_t i = 0; i < parts.size(); ++i) {
    shift(i, base);
    base += int64_t(parts[i].size());
  }
  return base;
}

int32_t* Planner::loc(int w) {
  std::vector<int32_t>& v = loc_[w];
  if (v.empty()) v.assign(g_.N, -1);
  return v.data();
}

void Planner::drop_inactive() {
  const size_t n = act_.size();
  constexpr size_t kBlock = 16384;
  const size_t nb = (n + kBlock - 1) / kBlock;
  if (nb <= 1 || workers_ <= 1) {
    size_t w = 0;
    for (size_t i = 0; i < n; ++i)
      if (active_[act_[i]]) act_[w++] = act_[i];
    act_.resize(w);
    return;
  }
  // per block: the survivors' count; a prefix sum then gives each block its
  // place in the output (order kept)
  std::vector<size_t> cnt(nb + 1, 0);
  parallel_for(nb, 1, workers_, [&](size_t b, int) {
    size_t c = 0;
    for (size_t i = b * kBlock; i < std::min(n, (b + 1) * kBlock); ++i) c += active_[act_[i]] != 0;
    cnt[b + 1] = c;
  });
  for (size_t b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
  // (into the spare array, whose memory is kept: a new one each time was
  // most of the cost)
  std::vector<int32_t>& out = act_spare_;
  out.resize(cnt[nb]);
  parallel_for(nb, 1, workers_, [&](size_t b, int) {
    size_t w = cnt[b];
    for (size_t i = b * kBlock; i < std::min(n, (b + 1) * kBlock); ++i)
      if (active_[act_[i]]) out[w++] = act_[i];
  });
  act_.swap(out);
}

void Planner::adopt_level0(std::shared_ptr<const LevelPlan> p) {
  lv_[0].plan = p;
  lv_[0].res.assign(p->groups.size(), GroupRes{});
  if (int64_t(active0_.size()) == g_.N) {   // the tree's level 0 seen before
    active_ = active0_;
    act_ = act0_;
    return;
  }
  fill_act();
  for (const Cell& C : p->cells)
    for (int32_t d : C.p) active_[d] = 0;
  drop_inactive();
  active0_ = active_;
  act0_ = act_;
}

void Planner::fill_act() {
  act_.resize(g_.N);
  for (int64_t d = 0; d < g_.N; ++d) act_[d] = int32_t(d);
}

// ---------------------------------------------------------------------------
// Cells of level l
// ---------------------------------------------------------------------------
void Planner::plan_cells(int l) {
  if (l == 0) fill_act();
  auto lp = std::make_shared<LevelPlan>();
  build_cells(l, *lp);
  if (l == 0) building0_ = lp;
  lv_[l].plan = lp;
  lv_[l].res.clear();
  // cells are disjoint: each byte is written by one cell
  parallel_for(lp->cells.size(), 64, workers_, [&](size_t ci, int) {
    for (int32_t d : lp->cells[ci].p) active_[d] = 0;
  });
  drop_inactive();
  if (l == 0) {   // the state adopt_level0 restores for later factorizations
    active0_ = active_;
    act0_ = act_;
  }
}

void Planner::build_cells(int l, LevelPlan& lp) {
  PlanTimer tm("cells", l);
  const bool top = (l == g_.L);
  const int64_t B = top ? 1 : boxes_per_axis(g_, l);
  int64_t nbox = 1;
  for (int k = 0; k < g_.dim; ++k) nbox *= B;
  const auto interior = [&](int64_t d) { return top || sigma(d, l) == 0; };

  // Interiors bucketed by box, ascending inside each box.
  std::vector<int32_t> keyv(act_.size());
  parallel_for(act_.size(), 8192, workers_, [&](size_t i, int) {
    const int32_t d = act_[i];
    keyv[i] = interior(d) ? int32_t(box_of(d, l)) : -1;
  });
  tm.mark("keys");
  std::vector<int32_t> count, order;
  bucket_by_key(keyv, nbox, workers_, count, order);
  std::vector<int32_t> cell_of_box(nbox, -1);
  std::vector<int64_t> box_of_cell;
  for (int64_t b = 0; b < nbox; ++b) {
    if (count[b + 1] == count[b]) continue;
    cell_of_box[b] = int32_t(lp.cells.size());
    Cell c;
    c.cid = top ? -1 : b;
    int64_t bb = b, par = 0;
    for (int k = 0; k < g_.dim; ++k) {
      par += bb % B;
      bb /= B;
    }
    c.color = int32_t(par & 1);
    lp.cells.push_back(std::move(c));
    box_of_cell.push_back(b);
  }
  parallel_for(lp.cells.size(), 64, workers_, [&](size_t ci, int) {
    const int64_t b = box_of_cell[ci];
    std::vector<int32_t>& p = lp.cells[ci].p;
    p.resize(size_t(count[b + 1] - count[b]));
    for (int32_t j = count[b]; j < count[b + 1]; ++j) p[size_t(j - count[b])] = act_[order[j]];
  });

  tm.mark("buckets");
  // Children (level l-1 cells inside each box) and interior bases.
  std::vector<std::vector<int32_t>> kids(lp.cells.size()), gkids(lp.cells.size());
  if (l > 0) {
    const Level& prev = lv_[l - 1];
    const int64_t Bp = boxes_per_axis(g_, l - 1);
    // parents found in parallel, lists filled in order
    std::vector<int32_t> kpar(prev.cells().size()), gpar(prev.groups().size(), -1);
    parallel_for(kpar.size(), 256, workers_, [&](size_t ci, int) {
      int64_t pb = prev.cells()[ci].cid, parent_box = 0, mul = 1;
      for (int k = 0; k < g_.dim; ++k) {
        int64_t bk = pb % Bp;
        pb /= Bp;
        parent_box += (top ? 0 : (bk / 2)) * mul;
        mul *= B;
      }
      const int32_t pc = cell_of_box[parent_box];
      if (pc < 0) throw std::runtime_error("planner: parent box without interior");
      kpar[ci] = pc;
    });
    parallel_for(gpar.size(), 256, workers_, [&](size_t gi, int) {
      const auto& surv = prev.survivors(gi);
      if (surv.empty()) return;
      const int64_t d0 = surv[0];
      if (!interior(d0)) return;
      gpar[gi] = cell_of_box[box_of(d0, l)];
    });
    for (size_t ci = 0; ci < kpar.size(); ++ci) kids[kpar[ci]].push_back(int32_t(ci));
    for (size_t gi = 0; gi < gpar.size(); ++gi)
      if (gpar[gi] >= 0) gkids[gpar[gi]].push_back(int32_t(gi));
  }

  tm.mark("children");
  // Per cell (independent; maps are collected per cell and concatenated).
  std::vector<std::vector<int32_t>> cmaps(lp.cells.size());
  parallel_for(lp.cells.size(), 8, workers_, [&](size_t ci, int w) {
    int32_t* loc_ = loc(w);
    Cell& C = lp.cells[ci];
    std::vector<int32_t>& maps = cmaps[ci];
    // Front q^+: surviving fronts of the children that are not interior
    // here, plus active stencil neighbours of the interior.
    std::vector<int32_t> q;
    if (l > 0)
      for (int32_t k : kids[ci])
        for (int32_t z : lv_[l - 1].cells()[k].q)
          if (active_[z] && !interior(z)) q.push_back(z);
    for (int32_t d : C.p)
      for_neighbors(d, [&](int64_t z, int, bool) {
        if (active_[z] && !interior(z)) q.push_back(int32_t(z));
      });
    std::sort(q.begin(), q.end());
    q.erase(std::unique(q.begin(), q.end()), q.end());
    C.q.swap(q);

    const int32_t np = int32_t(C.p.size());
    for (int32_t i = 0; i < np; ++i) loc_[C.p[i]] = i;
    for (int32_t i = 0; i < int32_t(C.q.size()); ++i) loc_[C.q[i]] = np + i;

    if (l > 0) {
      const Level& prev = lv_[l - 1];
      for (int32_t k : kids[ci]) {
        const Cell& K = prev.cells()[k];
        Source s{SRC_CELL_U, l - 1, k, int32_t(K.q.size()), int64_t(maps.size()), 0};
        s.colmap = s.rowmap;
        for (int32_t z : K.q) {
          if (active_[z] && loc_[z] < 0)
            throw std::runtime_error("planner: child front unknown lost by its parent");
          maps.push_back(active_[z] ? loc_[z] : -1);
        }
        C.src.push_back(s);
      }
      for (int32_t gi : gkids[ci]) {
        const auto& surv = prev.survivors(gi);
        Source s{SRC_GROUP_BASE, l - 1, gi, int32_t(surv.size()), int64_t(maps.size()), 0};
        s.colmap = s.rowmap;
        for (int32_t z : surv) {
          if (loc_[z] < 0) throw std::runtime_error("planner: base unknown outside its cell");
          maps.push_back(loc_[z]);
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
        C.trips.push_back({loc_[d], loc_[z], link_ref(g_.N, up ? d : z, k)});
      });
    }
    for (int32_t d : C.p) loc_[d] = -1;
    for (int32_t d : C.q) loc_[d] = -1;
  });
  tm.mark("fronts");
  lp.maps.resize(concat_offsets(cmaps, [&](size_t i, int64_t base) {
    for (Source& s : lp.cells[i].src) {
      s.rowmap += base;
      s.colmap += base;
    }
  }));
  parallel_for(cmaps.size(), 64, workers_, [&](size_t i, int) {
    if (!lp.cells[i].src.empty())
      std::copy(cmaps[i].begin(), cmaps[i].end(), lp.maps.begin() + lp.cells[i].src[0].rowmap);
  });
  tm.mark("maps");
}

// ---------------------------------------------------------------------------
// Groups of level l+1/2
// ---------------------------------------------------------------------------
void Planner::plan_groups(int l) {
  // The level's cells were planned by plan_cells(l) into a plan this planner
  // created (level 0 too, unless it was adopted; adopted plans already hold
  // their groups).
  std::shared_ptr<LevelPlan> lp = std::const_pointer_cast<LevelPlan>(lv_[l].plan);
  if (l == 0 && !building0_) {
    lv_[0].res.assign(lp->groups.size(), GroupRes{});
    return;
  }
  lp->groups.clear();
  lp->gmaps.clear();
  build_groups(l, *lp);
  lv_[l].res.assign(lp->groups.size(), GroupRes{});
  if (l == 0) building0_.reset();
}

void Planner::build_groups(int l, LevelPlan& lp) {
  PlanTimer tm("groups", l);
  const int64_t B = boxes_per_axis(g_, l);
  int64_t nkey = g_.dim;
  for (int k = 0; k < g_.dim; ++k) nkey *= B;
  std::vector<int32_t> keyv(act_.size());
  parallel_for(act_.size(), 8192, workers_, [&](size_t i, int) {
    const int32_t d = act_[i];
    keyv[i] = sigma(d, l) == 1 ? int32_t(group_key(d, l)) : -1;
  });
  tm.mark("keys");
  std::vector<int32_t> count, order;
  bucket_by_key(keyv, nkey, workers_, count, order);
  std::vector<int32_t> group_of_key(nkey, -1);
  for (int64_t b = 0; b < nkey; ++b) {
    if (count[b + 1] == count[b]) continue;
    group_of_key[b] = int32_t(lp.groups.size());
    Group G;
    G.gid = b;
    lp.groups.push_back(std::move(G));
  }
  parallel_for(lp.groups.size(), 64, workers_, [&](size_t gi, int) {
    const int64_t b = lp.groups[gi].gid;
    std::vector<int32_t>& c = lp.groups[gi].c;
    c.resize(size_t(count[b + 1] - count[b]));
    for (int32_t j = count[b]; j < count[b + 1]; ++j) c[size_t(j - count[b])] = act_[order[j]];
  });

  tm.mark("buckets");
  // Which level-l fronts hold each unknown (at most two).
  // (in either order: the groups only use the set)
  const auto& cells = lp.cells;
  parallel_for(cells.size(), 16, workers_, [&](size_t ci, int) {
    for (int32_t z : cells[ci].q) {
      int32_t expect = -1;
      if (__atomic_compare_exchange_n(&own0_[z], &expect, int32_t(ci), false, __ATOMIC_RELAXED,
                                      __ATOMIC_RELAXED))
        continue;
      expect = -1;
      if (!__atomic_compare_exchange_n(&own1_[z], &expect, int32_t(ci), false, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED))
        throw std::runtime_error("planner: unknown in more than two fronts");
    }
  });
  tm.mark("owners");
  // Earlier bases that land in each group.
  std::vector<std::vector<int32_t>> gkids(lp.groups.size());
  if (l > 0) {
    // parents found in parallel, lists filled in order
    const Level& prev = lv_[l - 1];
    std::vector<int32_t> gpar(prev.groups().size(), -1);
    parallel_for(gpar.size(), 256, workers_, [&](size_t gi, int) {
      const auto& surv = prev.survivors(gi);
      if (surv.empty()) return;
      const int32_t d0 = surv[0];
      if (sigma(d0, l) != 1) return;
      const int32_t g = group_of_key[group_key(d0, l)];
      if (g < 0) throw std::runtime_error("planner: base without group");
      gpar[gi] = g;
    });
    for (size_t gi = 0; gi < gpar.size(); ++gi)
      if (gpar[gi] >= 0) gkids[gpar[gi]].push_back(int32_t(gi));
  }
  tm.mark("children");
  std::vector<std::vector<int32_t>> gm(lp.groups.size());
  parallel_for(lp.groups.size(), 16, workers_, [&](size_t gi, int w) {
    int32_t* loc_ = loc(w);
    std::vector<int32_t>& gmaps = gm[gi];
    Group& G = lp.groups[gi];
    const int32_t nc = int32_t(G.c.size());
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = i;
    std::vector<int32_t> adj, cn;
    for (int32_t d : G.c) {
      if (own0_[d] >= 0) adj.push_back(own0_[d]);
      if (own1_[d] >= 0) adj.push_back(own1_[d]);
    }
    std::sort(adj.begin(), adj.end());
    adj.erase(std::unique(adj.begin(), adj.end()), adj.end());
    for (int32_t ci : adj)
      for (int32_t z : cells[ci].q)
        if (loc_[z] < 0) cn.push_back(z);
    for (int32_t d : G.c)
      for_neighbors(d, [&](int64_t z, int, bool) {
        if (active_[z] && loc_[z] < 0) cn.push_back(int32_t(z));
      });
    std::sort(cn.begin(), cn.end());
    cn.erase(std::unique(cn.begin(), cn.end()), cn.end());
    G.cN.swap(cn);
    const int32_t nn = int32_t(G.cN.size());

    // Base formation: earlier bases and loose entries inside c (local in c).
    if (l > 0) {
      const Level& prev = lv_[l - 1];
      for (int32_t pg : gkids[gi]) {
        const auto& surv = prev.survivors(pg);
        Source s{SRC_GROUP_BASE, l - 1, pg, int32_t(surv.size()), int64_t(gmaps.size()), 0};
        s.colmap = s.rowmap;
        for (int32_t z : surv) {
          if (loc_[z] < 0) throw std::runtime_error("planner: base unknown outside its group");
          gmaps.push_back(loc_[z]);
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
        G.gtrips.push_back({int32_t(it - G.cN.begin()), loc_[d], link_ref(g_.N, up ? d : z, k)});
      });
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = -1;

    // Cell update blocks -> [c^N; c] x c.
    for (int32_t i = 0; i < nn; ++i) loc_[G.cN[i]] = i;
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = nn + i;
    for (int32_t ci : adj) {
      const Cell& C = cells[ci];
      Source s{SRC_CELL_U, l, ci, int32_t(C.q.size()), int64_t(gmaps.size()), 0};
      for (int32_t z : C.q) gmaps.push_back(loc_[z]);
      s.colmap = int64_t(gmaps.size());
      for (int32_t z : C.q) gmaps.push_back(loc_[z] >= nn ? loc_[z] - nn : -1);
      G.gsrc.push_back(s);
    }
    for (int32_t i = 0; i < nn; ++i) loc_[G.cN[i]] = -1;
    for (int32_t i = 0; i < nc; ++i) loc_[G.c[i]] = -1;
  });
  tm.mark("groups");
  std::vector<int64_t> gbase(lp.groups.size());
  lp.gmaps.resize(concat_offsets(gm, [&](size_t i, int64_t base) {
    gbase[i] = base;
    Group& G = lp.groups[i];
    for (Source& s : G.bsrc) {
      s.rowmap += base;
      s.colmap += base;
    }
    for (Source& s : G.gsrc) {
      s.rowmap += base;
      s.colmap += base;
    }
  }));
  parallel_for(gm.size(), 64, workers_, [&](size_t i, int) {
    std::copy(gm[i].begin(), gm[i].end(), lp.gmaps.begin() + gbase[i]);
  });
  tm.mark("maps");
  parallel_for(cells.size(), 16, workers_, [&](size_t ci, int) {
    for (int32_t z : cells[ci].q) {
      __atomic_store_n(&own0_[z], -1, __ATOMIC_RELAXED);
      __atomic_store_n(&own1_[z], -1, __ATOMIC_RELAXED);
    }
  });
  tm.mark("owner reset");
}

void Planner::set_skeleton(int l, int gi, int k, const int32_t* sk_pos) {
  const Group& G = lv_[l].plan->groups.at(gi);
  GroupRes& R = lv_[l].res.at(gi);
  const int32_t nc = int32_t(G.c.size());
  R.k = k;
  R.sk.clear();
  R.rd.clear();
  if (k >= nc) {
    R.skel = false;
    R.k = nc;
    return;
  }
  R.skel = true;
  std::vector<uint8_t> is_sk(nc, 0);
  for (int i = 0; i < k; ++i) is_sk.at(sk_pos[i]) = 1;
  for (int32_t i = 0; i < nc; ++i) (is_sk[i] ? R.sk : R.rd).push_back(G.c[i]);
}

void Planner::set_skeletons(int l, const int32_t* ks, const int32_t* pos, size_t stride) {
  Level& lev = lv_[l];
  const std::vector<Group>& groups = lev.plan->groups;
  parallel_for(groups.size(), 32, workers_, [&](size_t gi, int) {
    const Group& G = groups[gi];
    GroupRes& R = lev.res.at(gi);
    const int32_t nc = int32_t(G.c.size());
    const int k = ks[gi];
    R.sk.clear();
    R.rd.clear();
    if (k >= nc) {
      R.skel = false;
      R.k = nc;
      return;
    }
    if (k < 0) throw std::runtime_error("negative rank");
    R.skel = true;
    R.k = k;
    // skeleton positions in increasing order, then both lists in the order
    // of c (as set_skeleton makes them)
    std::vector<int32_t>& sp = R.sk;
    sp.assign(pos + gi * stride, pos + gi * stride + k);
    std::sort(sp.begin(), sp.end());
    for (int i = 0; i < k; ++i)
      if (sp[i] < 0 || sp[i] >= nc || (i > 0 && sp[i] == sp[i - 1]))
        throw std::runtime_error("invalid skeleton position");
    R.rd.reserve(size_t(nc - k));
    int j = 0;
    for (int32_t i = 0; i < nc; ++i) {
      if (j < k && sp[j] == i) {
        sp[j++] = G.c[i];
      } else {
        R.rd.push_back(G.c[i]);
      }
    }
  });
}

void Planner::finish_groups(int l) {
  PlanTimer tm("finish", l);
  const Level& lev = lv_[l];
  // groups are disjoint: each byte is written by one group
  parallel_for(lev.groups().size(), 64, workers_, [&](size_t gi, int) {
    for (int32_t d : lev.groups()[gi].c) grouped_[d] = 1;
    if (lev.res[gi].skel)
      for (int32_t d : lev.res[gi].rd) active_[d] = 0;
  });
  tm.mark("marks");
  drop_inactive();
  tm.mark("compaction");
}

void plan_parallel(size_t n, size_t grain, const std::function<void(size_t)>& f) {
  parallel_for(n, grain, PlanPool::get().size(), [&](size_t i, int) { f(i); });
}

void planning_begin() { Janitor::get().planning(1); }
void planning_end() { Janitor::get().planning(-1); }

void discard_planner(std::unique_ptr<Planner> p) {
  if (p) Janitor::get().discard(std::move(p));
}

}  // namespace hifde
