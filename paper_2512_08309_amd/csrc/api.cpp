// C-ABI of the lazy sampler: query planning (kappa and the dependency cone),
// the device cache of per-window contributions with LRU eviction, and the
// per-level execution order.
//
// A query J_t[R] (Alg. 1, Sec. 3.3) is served level by level:
//   plan   : for l = t, t+1, ...: I_l = kappa(R_l) (window-range algorithm of
//            the appendix, exact floor/ceil in int64); windows of I_l already
//            in the cache are reused (they are the processed set P_l), the
//            others are new; R_{l+1} = bounding region of the new windows,
//            whose inputs J_{l+1}[R_i] are needed.  Planning stops at the
//            first level without new windows, or at T (noise).
//   run    : from the deepest planned level up: build J_{l+1} on R_{l+1}
//            (seed noise at T, else the blend of level-(l+1) contributions),
//            run the new windows through the batched denoiser, whose output
//            epilogue stores V_i = W (x) Phi(J_{l+1}[R_i]) straight into the
//            cache slots.  All windows of one level form one batched round
//            (split only by workspace size), so a cold query needs at most
//            T - t rounds (Parallelization theorem).
//   output : J_t[R] = blend of the level-t contributions (0/0 := 0).
// Evicting a contribution also removes it from the processed set (Sec. 3.3),
// so it is simply recomputed when next needed: values never depend on cache
// state (seed consistency).
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <cmath>
#include <cstring>
#include <list>
#include <memory>
#include <unordered_map>

#include "../../include/td.h"
#include "plan.h"
#include "model.h"
#include "profile.h"

namespace td {
namespace {

struct Key {
  uint64_t seed;
  int32_t level;
  int64_t ix, iy;
  bool operator==(const Key& o) const {
    return seed == o.seed && level == o.level && ix == o.ix && iy == o.iy;
  }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = k.seed * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)k.level + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.ix * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.iy * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

// Device slab of fixed-size contribution slots.
class SlotPool {
 public:
  ~SlotPool() { release(); }
  void configure(size_t slot_floats) {
    release();
    slot_floats_ = slot_floats;
    per_chunk_ = std::max<size_t>(1, (size_t)(256u << 20) / (slot_floats * 4));
  }
  void release() {
    for (float* c : chunks_) (void)hipFree(c);
    chunks_.clear();
    free_.clear();
    total_ = 0;
  }
  float* ptr(uint32_t s) const { return chunks_[s / per_chunk_] + (size_t)(s % per_chunk_) * slot_floats_; }
  uint32_t take() {
    if (free_.empty()) {
      float* c = nullptr;
      TD_HIP(hipMalloc(&c, per_chunk_ * slot_floats_ * sizeof(float)));
      chunks_.push_back(c);
      for (size_t i = per_chunk_; i-- > 0;) free_.push_back((uint32_t)(total_ + i));
      total_ += per_chunk_;
    }
    uint32_t s = free_.back();
    free_.pop_back();
    return s;
  }
  void give(uint32_t s) { free_.push_back(s); }
  size_t slot_bytes() const { return slot_floats_ * sizeof(float); }

 private:
  size_t slot_floats_ = 0, per_chunk_ = 1, total_ = 0;
  std::vector<float*> chunks_;
  std::vector<uint32_t> free_;
};

struct Entry {
  uint32_t slot;
  int pins;
  std::list<Key>::iterator lru;
};

// Host staging (pinned) + device mirror for per-query metadata.
class Arena {
 public:
  ~Arena() { release(); }
  void release() {
    if (h_) (void)hipHostFree(h_);
    if (d_) (void)hipFree(d_);
    h_ = nullptr;
    d_ = nullptr;
    cap_ = off_ = 0;
  }
  void reset() { off_ = 0; }
  // Make room for `bytes` more of reservations.  Called where no reservation
  // is outstanding (each was copied and its kernels enqueued), so growing
  // only has to wait for the device: then the old buffers are no longer read
  // and the new ones start empty.
  void ensure(size_t bytes) {
    if (off_ + bytes <= cap_) return;
    TD_HIP(hipDeviceSynchronize());
    const size_t want = std::max<size_t>(std::max(bytes, 2 * cap_), 1 << 20);
    release();
    TD_HIP(hipHostMalloc((void**)&h_, want, hipHostMallocDefault));
    TD_HIP(hipMalloc((void**)&d_, want));
    cap_ = want;
  }
  // Reserve n bytes; returns the host and device addresses.
  std::pair<char*, char*> reserve(size_t n) {
    n = (n + 255) / 256 * 256;
    if (off_ + n > cap_) {
      TD_CHECK(off_ == 0, -2, "metadata arena overflow within a query");
      ensure(n);
    }
    auto r = std::make_pair(h_ + off_, d_ + off_);
    off_ += n;
    return r;
  }

 private:
  char* h_ = nullptr;
  char* d_ = nullptr;
  size_t cap_ = 0, off_ = 0;
};

struct Level {
  int t;
  Region region;      // R_t
  Kappa k;            // kappa(R_t)
  std::vector<std::pair<int64_t, int64_t>> fresh;  // new windows (ix, iy), canonical order
  Region in_region{}; // bbox of the new windows = region at t+1
};

}  // namespace
}  // namespace td

struct td_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::unique_ptr<td::Model> model;
  td::SlotPool pool;
  std::unordered_map<td::Key, td::Entry, td::KeyHash> map;
  std::list<td::Key> lru;  // front = most recent
  size_t budget = (size_t)8 << 30;
  int batch = 0;           // 0 = automatic
  td_cache_stats_t stats{};
  std::string err;
  td::Arena arena;
  hipEvent_t done = nullptr;
  bool pending = false;
  float* canvas = nullptr;
  size_t canvas_cap = 0;
  float* tmp = nullptr;
  size_t tmp_cap = 0;
  float* dec = nullptr;
  size_t dec_cap = 0;
  float* outbuf = nullptr;
  size_t outbuf_cap = 0;
  float* gath = nullptr;      // batched window inputs of sample_latent_multi
  size_t gath_cap = 0;
  float* fb = nullptr;        // the judge's J_0 on the hull of fallen-back windows
  size_t fb_cap = 0;
  std::unique_ptr<td::Profiler> prof;
  // hierarchy: the parent whose final latent conditions this model, the
  // children it conditions, and a generation that changes with the values
  // this context produces (weights, precision)
  td_ctx* parent = nullptr;
  std::vector<td_ctx*> children;
  uint64_t gen = 1, parent_gen = 0;
  float* cond = nullptr;      // parent latent of the current query, [h][w][Cc]
  size_t cond_cap = 0;
  hipEvent_t xev = nullptr;   // orders this stream and the parent's
  hipEvent_t uev = nullptr;   // orders a caller's stream and this one
  // consistency sampling: the teacher whose one-step estimate judges ours
  td_ctx* judge = nullptr;
  std::vector<td_ctx*> judged_by;
  uint64_t judge_gen = 0;
  float judge_thr = 0.f;
  unsigned long long* d_fallbacks = nullptr;   // device counter
  uint64_t fallbacks_base = 0;
};

namespace td {
namespace {

void grow(float*& p, size_t& cap, size_t n) {
  if (n <= cap) return;
  size_t want = std::max(n, cap * 3 / 2);
  TD_HIP(hipDeviceSynchronize());
  if (p) TD_HIP(hipFree(p));
  p = nullptr;
  cap = 0;
  TD_HIP(hipMalloc(&p, want * sizeof(float)));
  cap = want;
}

void need_model(td_ctx* c) { TD_CHECK(c->model, TD_E_STATE, "no weights loaded"); }

// Windows that took the judge's estimate since the context was made.
uint64_t read_fallbacks(td_ctx* c) {
  if (!c->d_fallbacks) return 0;
  unsigned long long v = 0;
  TD_HIP(hipSetDevice(c->device));
  TD_HIP(hipStreamSynchronize(c->stream));
  TD_HIP(hipMemcpy(&v, c->d_fallbacks, sizeof(v), hipMemcpyDeviceToHost));
  return (uint64_t)v;
}

// Drops every cached contribution (none may be pinned by a query in flight).
void drop_cache(td_ctx* c) {
  for (auto& kv : c->map) c->pool.give(kv.second.slot);
  c->map.clear();
  c->lru.clear();
  c->stats.bytes_used = 0;
}

Region region_union(const Region& a, const Region& b) {
  if (a.w <= 0) return b;
  const int64_t x0 = std::min(a.x0, b.x0), y0 = std::min(a.y0, b.y0);
  const int64_t x1 = std::max(a.x0 + a.w, b.x0 + b.w), y1 = std::max(a.y0 + a.h, b.y0 + b.h);
  return Region{x0, y0, x1 - x0, y1 - y0};
}

void judge_fallback(void* user, const FallbackReq* req, int n, float* out, hipStream_t st);

void check_judge(td_ctx* c, bool may_clear) {
  td_ctx* j = c->judge;
  if (!j) {
    c->model->set_judge(nullptr, 0.f, nullptr);
    return;
  }
  const ModelDesc& d = c->model->d;
  TD_CHECK(d.consistency, TD_E_STATE, "a judge applies to consistency sampling only");
  TD_CHECK(j->model, TD_E_STATE, "the judge context has no weights");
  const ModelDesc& t = j->model->d;
  TD_CHECK(t.C == d.C && t.H == d.H && t.S == d.S && t.O == d.O, TD_E_STATE,
           "judge and student must share channels and window layout");
  TD_CHECK(!t.Cc || (t.Cc == d.Cc && t.cond_factor == d.cond_factor), TD_E_STATE,
           "a conditioned judge needs the student's conditioning");
  if (c->judge_gen != j->gen) {
    TD_CHECK(may_clear || c->map.empty(), TD_E_STATE, "the judge model changed while queries are in flight");
    drop_cache(c);
    c->judge_gen = j->gen;
  }
  c->model->set_judge(j->model.get(), c->judge_thr, c->d_fallbacks, judge_fallback, c);
}

// Orders the judge's stream around work on c's stream that uses the judge's
// model (before: after the judge's own work; after: the judge waits).
void judge_fence(td_ctx* c, bool before) {
  td_ctx* j = c->judge;
  if (!j) return;
  if (before) {
    TD_HIP(hipEventRecord(j->xev, j->stream));
    TD_HIP(hipStreamWaitEvent(c->stream, j->xev, 0));
  } else {
    TD_HIP(hipEventRecord(j->xev, c->stream));
    TD_HIP(hipStreamWaitEvent(j->stream, j->xev, 0));
  }
}

// A conditioned model needs its parent; its cache is only valid for the
// parent's current generation.  `may_clear`: no query holds pins.  Also
// refreshes the consistency judge.
void check_parent(td_ctx* c, bool may_clear) {
  check_judge(c, may_clear);
  const ModelDesc& d = c->model->d;
  if (!d.Cc) return;
  td_ctx* p = c->parent;
  TD_CHECK(p && p->model, TD_E_STATE, "conditioned model: link a parent with td_set_conditioning");
  TD_CHECK(p->model->d.C == d.Cc, TD_E_STATE, "parent channels differ from the conditioning channels");
  if (c->parent_gen != p->gen) {
    TD_CHECK(may_clear || c->map.empty(), TD_E_STATE, "the parent model changed while queries are in flight");
    drop_cache(c);
    c->parent_gen = p->gen;
  }
}

// Parent-resolution cover of a child region.
Region parent_region(const ModelDesc& d, const Region& r) {
  const int64_t f = d.cond_factor;
  const int64_t x0 = floordiv64(r.x0, f), y0 = floordiv64(r.y0, f);
  return Region{x0, y0, floordiv64(r.x0 + r.w - 1, f) - x0 + 1, floordiv64(r.y0 + r.h - 1, f) - y0 + 1};
}

void touch(td_ctx* c, Entry& e, const Key&) {
  c->lru.splice(c->lru.begin(), c->lru, e.lru);   // iterators stay valid
}

void evict_to_budget(td_ctx* c) {
  size_t sb = c->pool.slot_bytes();
  auto it = c->lru.end();
  while (c->map.size() * sb > c->budget && it != c->lru.begin()) {
    --it;
    auto m = c->map.find(*it);
    if (m->second.pins > 0) continue;
    c->pool.give(m->second.slot);
    c->map.erase(m);
    it = c->lru.erase(it);
    c->stats.evictions++;
  }
  c->stats.bytes_used = c->map.size() * sb;
}

void unpin_level(td_ctx* c, uint64_t seed, const Level& lv) {
  if (lv.k.empty) return;
  for (int64_t iy = lv.k.iy0; iy <= lv.k.iy1; ++iy)
    for (int64_t ix = lv.k.ix0; ix <= lv.k.ix1; ++ix) {
      auto m = c->map.find(Key{seed, lv.t, ix, iy});
      if (m != c->map.end() && m->second.pins > 0) m->second.pins--;
    }
}

// Device pointer grid of level lv's contributions over lv.k (all present).
const float* const* pointer_grid(td_ctx* c, Arena& arena, uint64_t seed, const Level& lv) {
  size_t n = (size_t)lv.k.count();
  auto hd = arena.reserve(n * sizeof(float*));
  const float** h = (const float**)hd.first;
  size_t i = 0;
  for (int64_t iy = lv.k.iy0; iy <= lv.k.iy1; ++iy)
    for (int64_t ix = lv.k.ix0; ix <= lv.k.ix1; ++ix) {
      auto m = c->map.find(Key{seed, lv.t, ix, iy});
      TD_CHECK(m != c->map.end(), TD_E_DEVICE, "internal: contribution missing from cache");
      h[i++] = c->pool.ptr(m->second.slot);
    }
  TD_HIP(hipMemcpyAsync(hd.second, hd.first, n * sizeof(float*), hipMemcpyHostToDevice, c->stream));
  return (const float* const*)hd.second;
}

void blend_into(td_ctx* c, Arena& arena, uint64_t seed, const Level& lv, const Region& r, int layout, float* out) {
  const ModelDesc& d = c->model->d;
  const float* const* grid = pointer_grid(c, arena, seed, lv);
  int64_t bx = lv.k.ix0 * d.S + d.O, by = lv.k.iy0 * d.S + d.O;
  WinGeom g{d.H, d.S, d.C};
  launch_blend(c->stream, g, (int)(r.x0 - bx), (int)(r.y0 - by), (int)r.w, (int)r.h, (int)lv.k.nx(),
               (int)lv.k.ny(), grid, c->model->w1d(), layout, out);
  if (d.consistency) {
    // level t came from step K-t-1: its state is re-noised to sigma_{K-t}
    // with fresh noise on counter word K-t (zero at the final level)
    const int kn = d.K - lv.t;
    if (d.sched[kn] > 0)
      launch_noise(c->stream, seed, r.x0, r.y0, (int)r.w, (int)r.h, d.C, (uint32_t)kn, (float)d.sched[kn], layout,
                   out, 1);
  }
}

// Windows per denoiser launch.  4-channel networks: as many as a 32 GB
// workspace holds, at most 1024 (measured on the 8192^2 cold query: 1024
// windows 3,380 window-denoises/s, 768 3,370, 512 3,357; the deepest level's
// launches then fill the chip twice instead of once).  Others: a 16 GB
// workspace, at most 4096.  The workspace is sized for this batch at a
// context's first query, so the budget is per live context.
int auto_batch(td_ctx* c) {
  if (c->batch > 0) return c->batch;
  size_t per = c->model->workspace_bytes_per_window();
  if (!per) return 1 << 20;
  const bool four = c->model->d.C == 4;
  size_t b = ((size_t)(four ? 32 : 16) << 30) / per;
  return (int)std::max<size_t>(1, std::min<size_t>(b, four ? 1024 : 4096));
}

void check_region(int64_t x0, int64_t y0, int64_t w, int64_t h) {
  const int64_t lim = (1LL << 31) - (1LL << 22);
  TD_CHECK(w >= 1 && h >= 1 && w <= (1 << 20) && h <= (1 << 20) && w * h <= (1LL << 26), TD_E_INVAL,
           "region sides must be in [1, 2^20] and its area at most 2^26 pixels");
  TD_CHECK(x0 > -lim && y0 > -lim && x0 + w < lim && y0 + h < lim, TD_E_INVAL, "region coordinates out of range");
}

void sample_latent(td_ctx* c, Arena& arena, uint64_t seed, Region r, int level, int layout, float* dev_out);

// The parent's J_0 on the parent-resolution cover of `hull` (child pixels),
// written to dst ([h][w][Cc], child-owned); rc receives the parent region.
// The parent runs on its own stream (and cache) after everything already
// enqueued on the child's.  Without `done` the child's later work waits for
// it; with `done` the completion is recorded there and the caller makes the
// child wait before it reads dst.
void sample_parent(td_ctx* c, Arena& arena, uint64_t seed, const Region& hull, float* dst, Region* rc,
                   hipEvent_t done = nullptr) {
  td_ctx* p = c->parent;
  *rc = parent_region(c->model->d, hull);
  check_region(rc->x0, rc->y0, rc->w, rc->h);
  TD_CHECK(p->device == c->device, TD_E_STATE, "parent and child must share a device");
  check_parent(p, true);
  TD_HIP(hipEventRecord(c->xev, c->stream));
  TD_HIP(hipStreamWaitEvent(p->stream, c->xev, 0));
  sample_latent(p, arena, seed, *rc, 0, 0, dst);
  if (done) {
    TD_HIP(hipEventRecord(done, p->stream));
  } else {
    TD_HIP(hipEventRecord(c->xev, p->stream));
    TD_HIP(hipStreamWaitEvent(c->stream, c->xev, 0));
  }
}

// One region of a multi-region query: J_0 of (seed, r) into dst, [h][w][C].
struct RegionJob {
  uint64_t seed;
  Region r;
  float* dst;
};

void sample_latent_multi(td_ctx* c, Arena& arena, const std::vector<RegionJob>& jobs);

// The parent latents of several child queries (seed, hull of new windows,
// destination), sampled together on the parent's stream after everything
// already enqueued on the child's; rcs receives the parent regions.
void sample_parents(td_ctx* c, Arena& arena, const std::vector<RegionJob>& hulls, std::vector<Region>* rcs) {
  td_ctx* p = c->parent;
  TD_CHECK(p->device == c->device, TD_E_STATE, "parent and child must share a device");
  check_parent(p, true);
  std::vector<RegionJob> jobs;
  rcs->clear();
  for (const RegionJob& h : hulls) {
    const Region rc = parent_region(c->model->d, h.r);
    check_region(rc.x0, rc.y0, rc.w, rc.h);
    rcs->push_back(rc);
    jobs.push_back(RegionJob{h.seed, rc, h.dst});
  }
  TD_HIP(hipEventRecord(c->xev, c->stream));
  TD_HIP(hipStreamWaitEvent(p->stream, c->xev, 0));
  sample_latent_multi(p, arena, jobs);
}

// Conditioning windows of a batch: window j (index (ix, iy)) reads the
// parent canvas whose origin in child pixels is (fx, fy).
void cond_batch(td_ctx* c, Arena& arena, const CondSrc* hsrc, int nb) {
  const ModelDesc& d = c->model->d;
  auto cs = arena.reserve((size_t)nb * sizeof(CondSrc));
  std::memcpy(cs.first, hsrc, (size_t)nb * sizeof(CondSrc));
  TD_HIP(hipMemcpyAsync(cs.second, cs.first, (size_t)nb * sizeof(CondSrc), hipMemcpyHostToDevice, c->stream));
  launch_cond_gather(c->stream, (const CondSrc*)cs.second, nb, d.H, d.Cc, d.cond_factor, c->model->cond_buffer());
}

CondSrc cond_src(const ModelDesc& d, const float* base, int64_t pitch, int64_t fx, int64_t fy, int64_t ix,
                 int64_t iy) {
  CondSrc q{};
  q.base = base;
  q.pitch = (int)pitch;
  const int64_t ox = ix * d.S + d.O - fx, oy = iy * d.S + d.O - fy;
  TD_CHECK(ox >= 0 && oy >= 0 && ox < (1LL << 30) && oy < (1LL << 30), TD_E_DEVICE,
           "internal: window outside its conditioning canvas");
  q.offx = (int)ox;
  q.offy = (int)oy;
  return q;
}

// J_level on region r written to dev_out (layout 0: [h][w][C], 1: [C][h][w]).
void sample_latent_body(td_ctx* c, Arena& arena, uint64_t seed, Region r, int level, int layout, float* dev_out) {
  const ModelDesc& d = c->model->d;
  hipStream_t st = c->stream;
  c->stats.queries++;
  if (level == d.T) {
    launch_noise(st, seed, r.x0, r.y0, (int)r.w, (int)r.h, d.C, d.noise_step, (float)d.sched[0], layout, dev_out);
    return;
  }
  // ---- plan
  std::vector<Level> levels;
  Region R = r;
  for (int t = level; t < d.T; ++t) {
    Level lv;
    lv.t = t;
    lv.region = R;
    lv.k = kappa(R, d.H, d.S, d.O);
    if (!lv.k.empty) {
      TD_CHECK(lv.k.count() <= (1LL << 26), TD_E_INVAL, "query too large");
      int64_t mnx = INT64_MAX, mxx = INT64_MIN, mny = INT64_MAX, mxy = INT64_MIN;
      for (int64_t iy = lv.k.iy0; iy <= lv.k.iy1; ++iy)
        for (int64_t ix = lv.k.ix0; ix <= lv.k.ix1; ++ix) {
          Key key{seed, t, ix, iy};
          auto m = c->map.find(key);
          if (m != c->map.end()) {
            m->second.pins++;
            touch(c, m->second, key);
            c->stats.hits++;
          } else {
            lv.fresh.push_back({ix, iy});
            mnx = std::min(mnx, ix);
            mxx = std::max(mxx, ix);
            mny = std::min(mny, iy);
            mxy = std::max(mxy, iy);
          }
        }
      if (!lv.fresh.empty())
        lv.in_region = Region{mnx * d.S + d.O, mny * d.S + d.O, (mxx - mnx) * d.S + d.H, (mxy - mny) * d.S + d.H};
    }
    levels.push_back(lv);
    if (lv.k.empty || lv.fresh.empty()) break;
    R = lv.in_region;
  }
  // ---- conditioning: the parent's latent under every new window
  Region rc{};
  if (d.Cc) {
    Region hull{0, 0, 0, 0};
    for (const Level& lv : levels)
      if (!lv.fresh.empty()) hull = region_union(hull, lv.in_region);
    if (hull.w > 0) {
      const Region pr = parent_region(d, hull);
      grow(c->cond, c->cond_cap, (size_t)pr.w * pr.h * d.Cc);
      sample_parent(c, arena, seed, hull, c->cond, &rc);
    }
  }
  // ---- run, deepest level first
  const int maxb = auto_batch(c);
  size_t meta = 65536;
  for (const Level& lv : levels) {
    meta += (size_t)lv.k.count() * sizeof(float*) + 256;
    size_t nbat = (lv.fresh.size() + maxb - 1) / maxb;
    meta += lv.fresh.size() * (4 * sizeof(int) + sizeof(float*) + sizeof(CondSrc)) + nbat * 4 * 256;
  }
  arena.ensure(meta);
  c->model->ensure_workspace(std::min<int>(maxb, 1 << 20));
  for (int i = (int)levels.size() - 1; i >= 0; --i) {
    Level& lv = levels[i];
    if (lv.k.empty || lv.fresh.empty()) continue;
    const Region& cr = lv.in_region;
    size_t cn = (size_t)cr.w * cr.h * d.C;
    grow(c->canvas, c->canvas_cap, cn);
    const int tn = lv.t + 1;
    if (tn == d.T) {
      launch_noise(st, seed, cr.x0, cr.y0, (int)cr.w, (int)cr.h, d.C, d.noise_step, (float)d.sched[0], 0,
                   c->canvas);
    } else {
      const Level& up = levels[i + 1];
      if (up.k.empty) launch_fill(st, c->canvas, cn, 0.f);
      else blend_into(c, arena, seed, up, cr, 0, c->canvas);
      unpin_level(c, seed, up);
    }
    // new windows -> slots, then batched denoiser rounds
    const size_t nf = lv.fresh.size();
    std::vector<uint32_t> slots(nf);
    for (size_t j = 0; j < nf; ++j) {
      Key key{seed, lv.t, lv.fresh[j].first, lv.fresh[j].second};
      slots[j] = c->pool.take();
      c->lru.push_front(key);
      c->map[key] = Entry{slots[j], 1, c->lru.begin()};
    }
    c->stats.misses += nf;
    c->stats.denoiser_evals += (uint64_t)nf * c->model->level_steps(lv.t);
    if (lv.t < 64) c->stats.windows_evaluated[lv.t] += nf;
    for (size_t b0 = 0; b0 < nf; b0 += (size_t)maxb) {
      int nb = (int)std::min<size_t>(maxb, nf - b0);
      auto o = arena.reserve((size_t)nb * 2 * sizeof(int));
      auto w = arena.reserve((size_t)nb * 2 * sizeof(int));
      auto s = arena.reserve((size_t)nb * sizeof(float*));
      int* ho = (int*)o.first;
      int* hw = (int*)w.first;
      float** hs = (float**)s.first;
      for (int j = 0; j < nb; ++j) {
        auto ij = lv.fresh[b0 + j];
        ho[2 * j] = (int)(ij.first * d.S + d.O - cr.x0);
        ho[2 * j + 1] = (int)(ij.second * d.S + d.O - cr.y0);
        hw[2 * j] = (int)ij.first;
        hw[2 * j + 1] = (int)ij.second;
        hs[j] = c->pool.ptr(slots[b0 + j]);
      }
      TD_HIP(hipMemcpyAsync(o.second, o.first, (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, st));
      TD_HIP(hipMemcpyAsync(w.second, w.first, (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, st));
      TD_HIP(hipMemcpyAsync(s.second, s.first, (size_t)nb * sizeof(float*), hipMemcpyHostToDevice, st));
      WindowBatch wb;
      wb.canvas = c->canvas;
      wb.canvas_w = (int)cr.w;
      wb.d_origins = (const int*)o.second;
      wb.d_widx = (const int*)w.second;
      wb.d_slots = (float* const*)s.second;
      wb.n = nb;
      wb.mode = 0;
      wb.h_widx = hw;
      wb.seed = seed;
      if (d.Cc) {
        std::vector<CondSrc> cs(nb);
        for (int j = 0; j < nb; ++j)
          cs[j] = cond_src(d, c->cond, rc.w, rc.x0 * d.cond_factor, rc.y0 * d.cond_factor, lv.fresh[b0 + j].first,
                           lv.fresh[b0 + j].second);
        cond_batch(c, arena, cs.data(), nb);
        wb.cond = c->model->cond_buffer();
      }
      c->model->run_level(st, wb, lv.t);
      c->stats.batches++;
    }
    evict_to_budget(c);
  }
  // ---- output
  const Level& top = levels[0];
  if (top.k.empty) {
    launch_fill(st, dev_out, (size_t)r.w * r.h * d.C, 0.f);
  } else {
    blend_into(c, arena, seed, top, r, layout, dev_out);
    unpin_level(c, seed, top);
  }
  evict_to_budget(c);
}

// J_0 of several regions (unconditioned models): each region's cone is
// planned as in sample_latent, but a window shared by several cones is
// evaluated once (the first region claims it; the others find it in the
// cache map and only pin it), and every level's new windows of all regions
// are gathered from their regions' canvases into shared batches.  Window
// values do not depend on the batch they run in, so each result equals the
// region's own sample_latent.
void sample_latent_multi_body(td_ctx* c, Arena& arena, const std::vector<RegionJob>& jobs) {
  const ModelDesc& d = c->model->d;
  TD_CHECK(d.Cc == 0, TD_E_STATE, "internal: batched regions of a conditioned model");
  hipStream_t st = c->stream;
  const int nr = (int)jobs.size();
  if (!nr) return;
  // ---- plan: levels[i][t] for region i; fresh windows enter the map now
  std::vector<std::vector<Level>> levels(nr);
  std::vector<std::vector<std::vector<uint32_t>>> slots(nr);
  int tmax = -1;
  size_t meta = 65536, nfresh = 0;
  for (int i = 0; i < nr; ++i) {
    c->stats.queries++;
    Region R = jobs[i].r;
    for (int t = 0; t < d.T; ++t) {
      Level lv;
      lv.t = t;
      lv.region = R;
      lv.k = kappa(R, d.H, d.S, d.O);
      std::vector<uint32_t> sl;
      if (!lv.k.empty) {
        TD_CHECK(lv.k.count() <= (1LL << 26), TD_E_INVAL, "query too large");
        int64_t mnx = INT64_MAX, mxx = INT64_MIN, mny = INT64_MAX, mxy = INT64_MIN;
        for (int64_t iy = lv.k.iy0; iy <= lv.k.iy1; ++iy)
          for (int64_t ix = lv.k.ix0; ix <= lv.k.ix1; ++ix) {
            Key key{jobs[i].seed, t, ix, iy};
            auto m = c->map.find(key);
            if (m != c->map.end()) {
              m->second.pins++;
              touch(c, m->second, key);
              c->stats.hits++;
              continue;
            }
            const uint32_t slot = c->pool.take();
            c->lru.push_front(key);
            c->map[key] = Entry{slot, 1, c->lru.begin()};
            sl.push_back(slot);
            lv.fresh.push_back({ix, iy});
            mnx = std::min(mnx, ix);
            mxx = std::max(mxx, ix);
            mny = std::min(mny, iy);
            mxy = std::max(mxy, iy);
          }
        if (!lv.fresh.empty())
          lv.in_region = Region{mnx * d.S + d.O, mny * d.S + d.O, (mxx - mnx) * d.S + d.H, (mxy - mny) * d.S + d.H};
        meta += (size_t)lv.k.count() * sizeof(float*) + 256;
      }
      nfresh += lv.fresh.size();
      const bool stop = lv.k.empty || lv.fresh.empty();
      if (!stop) tmax = std::max(tmax, t);
      levels[i].push_back(std::move(lv));
      slots[i].push_back(std::move(sl));
      if (stop) break;
      R = levels[i].back().in_region;
    }
  }
  const int maxb = auto_batch(c);
  meta += nfresh * (3 * sizeof(int) + 2 * sizeof(float*)) + (nfresh / maxb + 2 * (tmax + 2)) * 5 * 256;
  arena.ensure(meta);
  c->model->ensure_workspace(std::min<int>(maxb, 1 << 20));
  const size_t per = (size_t)d.H * d.H * d.C;
  // ---- run, deepest level first
  for (int t = tmax; t >= 0; --t) {
    // canvases of this level, one per region with new windows here
    std::vector<size_t> off(nr, 0);
    size_t total = 0;
    for (int i = 0; i < nr; ++i)
      if (t < (int)levels[i].size() && !levels[i][t].fresh.empty()) {
        off[i] = total;
        const Region& cr = levels[i][t].in_region;
        total += (size_t)cr.w * cr.h * d.C;
      }
    if (!total) continue;
    grow(c->canvas, c->canvas_cap, total);
    std::vector<std::pair<int, size_t>> work;   // (region, index into its fresh list)
    for (int i = 0; i < nr; ++i) {
      if (t >= (int)levels[i].size() || levels[i][t].fresh.empty()) continue;
      Level& lv = levels[i][t];
      const Region& cr = lv.in_region;
      float* canvas = c->canvas + off[i];
      if (t + 1 == d.T) {
        launch_noise(st, jobs[i].seed, cr.x0, cr.y0, (int)cr.w, (int)cr.h, d.C, d.noise_step, (float)d.sched[0], 0,
                     canvas);
      } else {
        const Level& up = levels[i][t + 1];
        if (up.k.empty) launch_fill(st, canvas, (size_t)cr.w * cr.h * d.C, 0.f);
        else blend_into(c, arena, jobs[i].seed, up, cr, 0, canvas);
        unpin_level(c, jobs[i].seed, up);
      }
      for (size_t j = 0; j < lv.fresh.size(); ++j) work.push_back({i, j});
      c->stats.misses += lv.fresh.size();
      c->stats.denoiser_evals += (uint64_t)lv.fresh.size() * c->model->level_steps(t);
      if (t < 64) c->stats.windows_evaluated[t] += lv.fresh.size();
    }
    grow(c->gath, c->gath_cap, (size_t)std::min<size_t>(work.size(), (size_t)maxb) * per);
    for (size_t b0 = 0; b0 < work.size(); b0 += (size_t)maxb) {
      const int nb = (int)std::min<size_t>(maxb, work.size() - b0);
      auto src = arena.reserve((size_t)nb * sizeof(float*));
      auto pit = arena.reserve((size_t)nb * sizeof(int));
      auto org = arena.reserve((size_t)nb * 2 * sizeof(int));
      auto wix = arena.reserve((size_t)nb * 2 * sizeof(int));
      auto slo = arena.reserve((size_t)nb * sizeof(float*));
      const float** hs = (const float**)src.first;
      int* hp = (int*)pit.first;
      int* ho = (int*)org.first;
      int* hw = (int*)wix.first;
      float** hsl = (float**)slo.first;
      for (int j = 0; j < nb; ++j) {
        const int i = work[b0 + j].first;
        const size_t f = work[b0 + j].second;
        const Level& lv = levels[i][t];
        const Region& cr = lv.in_region;
        const auto ij = lv.fresh[f];
        const int64_t ox = ij.first * d.S + d.O - cr.x0, oy = ij.second * d.S + d.O - cr.y0;
        hs[j] = c->canvas + off[i] + ((size_t)oy * cr.w + ox) * d.C;
        hp[j] = (int)cr.w;
        ho[2 * j] = 0;
        ho[2 * j + 1] = j * d.H;
        hw[2 * j] = (int)ij.first;
        hw[2 * j + 1] = (int)ij.second;
        hsl[j] = c->pool.ptr(slots[i][t][f]);
      }
      TD_HIP(hipMemcpyAsync(src.second, src.first, (size_t)nb * sizeof(float*), hipMemcpyHostToDevice, st));
      TD_HIP(hipMemcpyAsync(pit.second, pit.first, (size_t)nb * sizeof(int), hipMemcpyHostToDevice, st));
      TD_HIP(hipMemcpyAsync(org.second, org.first, (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, st));
      TD_HIP(hipMemcpyAsync(wix.second, wix.first, (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, st));
      TD_HIP(hipMemcpyAsync(slo.second, slo.first, (size_t)nb * sizeof(float*), hipMemcpyHostToDevice, st));
      launch_gather(st, (const float* const*)src.second, (const int*)pit.second, nb, d.H, d.C, c->gath);
      std::vector<uint64_t> seeds(nb);
      for (int j = 0; j < nb; ++j) seeds[j] = jobs[work[b0 + j].first].seed;
      WindowBatch wb;
      wb.canvas = c->gath;
      wb.canvas_w = d.H;
      wb.d_origins = (const int*)org.second;
      wb.d_widx = (const int*)wix.second;
      wb.d_slots = (float* const*)slo.second;
      wb.n = nb;
      wb.mode = 0;
      wb.h_widx = hw;
      wb.h_seeds = seeds.data();
      c->model->run_level(st, wb, t);
      c->stats.batches++;
    }
    evict_to_budget(c);
  }
  // ---- outputs
  for (int i = 0; i < nr; ++i) {
    const Level& top = levels[i][0];
    const Region& r = jobs[i].r;
    if (top.k.empty) {
      launch_fill(st, jobs[i].dst, (size_t)r.w * r.h * d.C, 0.f);
    } else {
      blend_into(c, arena, jobs[i].seed, top, r, 0, jobs[i].dst);
      unpin_level(c, jobs[i].seed, top);
    }
  }
  evict_to_budget(c);
}

// Latent apron of a full-resolution region (decode reads 17 latent px).
Region decode_apron(const ModelDesc& d, const Region& full) {
  const int R = d.blur_radius;
  int64_t xl = floordiv64(2 * full.x0 - 7, 16), xh = floordiv64(2 * (full.x0 + full.w - 1) - 7, 16) + 1;
  int64_t yl = floordiv64(2 * full.y0 - 7, 16), yh = floordiv64(2 * (full.y0 + full.h - 1) - 7, 16) + 1;
  return Region{xl - R - 1, yl - R - 1, xh - xl + 2 * R + 3, yh - yl + 2 * R + 3};
}

DecodeArgs decode_args(td_ctx* c, const float* latent, const Region& lat, const Region& full, float* out) {
  const ModelDesc& d = c->model->d;
  DecodeArgs a{};
  a.latent = latent;
  a.lx0 = lat.x0;
  a.ly0 = lat.y0;
  a.lw = (int)lat.w;
  a.lh = (int)lat.h;
  a.C = d.C;
  a.X0 = full.x0;
  a.Y0 = full.y0;
  a.W = (int)full.w;
  a.H = (int)full.h;
  a.out = out;
  a.sigma_low = (float)d.sigma_low;
  a.sigma_res = (float)d.sigma_res;
  a.taps = c->model->decode_taps();
  a.radius = d.blur_radius;
  a.atoms = c->model->decode_atoms();
  return a;
}

void decode_into(td_ctx* c, const float* latent, const Region& lat, const Region& full, float* out, hipStream_t st) {
  DecodeArgs a = decode_args(c, latent, lat, full, out);
  size_t wf = decode_work_floats(a);
  grow(c->dec, c->dec_cap, 2 * wf);
  a.work0 = c->dec;
  a.work1 = c->dec + wf;
  launch_decode(st, a);
}

// A query that fails part-way (an allocation, a launch, a rejected level)
// can leave windows pinned, or claimed in the map without their contribution
// having been written.  The cache only ever changes speed, not values, so it
// is dropped once the stream has drained instead of being repaired.
void abandon_cache(td_ctx* c) {
  (void)hipStreamSynchronize(c->stream);
  drop_cache(c);
}

void sample_latent(td_ctx* c, Arena& arena, uint64_t seed, Region r, int level, int layout, float* dev_out) {
  try {
    sample_latent_body(c, arena, seed, r, level, layout, dev_out);
  } catch (...) {
    abandon_cache(c);
    throw;
  }
}

void sample_latent_multi(td_ctx* c, Arena& arena, const std::vector<RegionJob>& jobs) {
  try {
    sample_latent_multi_body(c, arena, jobs);
  } catch (...) {
    abandon_cache(c);
    throw;
  }
}

// Fallback of a judged consistency model (Sec. 3.4 lets Phi be a few-step
// model; Sec. 5.3 distils the plain sampler into two steps, which then
// stands behind it): a flagged window takes the judge's plain sample J_0
// on the window's region, same seed, written to out[j] as [H][H][C].  It
// runs on the judge's stream and cache after everything enqueued on `st`,
// and `st` waits for it.  Windows of one seed are sampled as one region,
// their bounding box, when they fill at least a quarter of it (or the judge
// is conditioned); otherwise as one multi-region query of window regions.
void judge_fallback(void* user, const FallbackReq* req, int n, float* out, hipStream_t st) {
  td_ctx* c = static_cast<td_ctx*>(user);
  td_ctx* j = c->judge;
  TD_CHECK(j && j->model, TD_E_STATE, "internal: fallback without a judge");
  TD_CHECK(j->device == c->device, TD_E_STATE, "judge and student must share a device");
  const ModelDesc& d = c->model->d;
  const size_t per = (size_t)d.H * d.H * d.C;
  TD_HIP(hipEventRecord(c->xev, st));
  TD_HIP(hipStreamWaitEvent(j->stream, c->xev, 0));
  // the judge's own earlier work (and its metadata copies) has finished
  TD_HIP(hipStreamSynchronize(j->stream));
  j->arena.reset();
  check_parent(j, true);
  std::map<uint64_t, std::vector<int>> by_seed;
  for (int i = 0; i < n; ++i) by_seed[req[i].seed].push_back(i);
  std::vector<RegionJob> jobs;
  for (const auto& g : by_seed) {
    Region hull{0, 0, 0, 0};
    for (int i : g.second)
      hull = region_union(hull, Region{req[i].ix * d.S + d.O, req[i].iy * d.S + d.O, d.H, d.H});
    const bool whole = j->model->d.Cc || (int64_t)g.second.size() * d.H * d.H * 4 >= hull.w * hull.h;
    if (!whole) {
      for (int i : g.second)
        jobs.push_back(RegionJob{g.first, Region{req[i].ix * d.S + d.O, req[i].iy * d.S + d.O, d.H, d.H},
                                 out + (size_t)i * per});
      continue;
    }
    check_region(hull.x0, hull.y0, hull.w, hull.h);
    grow(c->fb, c->fb_cap, (size_t)hull.w * hull.h * d.C);
    sample_latent(j, j->arena, g.first, hull, 0, 0, c->fb);
    for (int i : g.second) {
      const size_t ox = (size_t)(req[i].ix * d.S + d.O - hull.x0), oy = (size_t)(req[i].iy * d.S + d.O - hull.y0);
      TD_HIP(hipMemcpy2DAsync(out + (size_t)i * per, (size_t)d.H * d.C * sizeof(float),
                              c->fb + (oy * hull.w + ox) * d.C, (size_t)hull.w * d.C * sizeof(float),
                              (size_t)d.H * d.C * sizeof(float), d.H, hipMemcpyDeviceToDevice, j->stream));
    }
  }
  if (!jobs.empty()) sample_latent_multi(j, j->arena, jobs);
  TD_HIP(hipEventRecord(j->xev, j->stream));
  TD_HIP(hipStreamWaitEvent(st, j->xev, 0));
}

void sample_any(td_ctx* c, uint64_t seed, int64_t x0, int64_t y0, int32_t w, int32_t h, int32_t level,
                float* dev_out, size_t out_len) {
  need_model(c);
  const ModelDesc& d = c->model->d;
  check_region(x0, y0, w, h);
  if (c->pending) {
    TD_HIP(hipEventSynchronize(c->done));
    c->pending = false;
  }
  c->arena.reset();
  check_parent(c, true);
  judge_fence(c, true);
  if (level == TD_LEVEL_HEIGHT) {
    TD_CHECK(out_len >= (size_t)w * h, TD_E_INVAL, "output buffer too small");
    Region full{x0, y0, w, h};
    Region lat = decode_apron(d, full);
    size_t n = (size_t)lat.w * lat.h * d.C;
    grow(c->tmp, c->tmp_cap, n);
    sample_latent(c, c->arena, seed, lat, 0, 0, c->tmp);
    decode_into(c, c->tmp, lat, full, dev_out, c->stream);
  } else {
    TD_CHECK(level >= 0 && level <= d.T, TD_E_INVAL, "level out of range");
    TD_CHECK(out_len >= (size_t)w * h * d.C, TD_E_INVAL, "output buffer too small");
    sample_latent(c, c->arena, seed, Region{x0, y0, w, h}, level, 1, dev_out);
  }
  c->stats.bytes_budget = c->budget;
  judge_fence(c, false);
  TD_HIP(hipEventRecord(c->done, c->stream));
  c->pending = true;
}

// Installs the context's profiler (if timing is on) for the launches of one call.
struct ProfScope {
  explicit ProfScope(td_ctx* c) { g_prof = c ? c->prof.get() : nullptr; }
  ~ProfScope() { g_prof = nullptr; }
};

template <class F>
td_status guarded(td_ctx* c, F&& f) {
  try {
    if (c) c->err.clear();
    ProfScope scope(c);
    f();
    return TD_OK;
  } catch (const Error& e) {
    if (c) c->err = e.msg;
    // a failed runtime call is reported once, here: clear it so that the
    // next launch check does not report it again
    if (e.status == TD_E_NOMEM || e.status == TD_E_DEVICE) (void)hipGetLastError();
    return (td_status)e.status;
  } catch (const std::bad_alloc&) {
    if (c) c->err = "host allocation failed";
    return TD_E_NOMEM;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return TD_E_DEVICE;
  }
}

}  // namespace
}  // namespace td

using namespace td;

extern "C" {

td_status td_create(int hip_device, td_ctx** out) {
  if (!out) return TD_E_INVAL;
  *out = nullptr;
  td_ctx* c = nullptr;
  try {
    c = new td_ctx();
  } catch (...) {
    return TD_E_NOMEM;
  }
  td_status s = guarded(c, [&] {
    int n = 0;
    TD_HIP(hipGetDeviceCount(&n));
    TD_CHECK(hip_device >= 0 && hip_device < n, TD_E_INVAL, "no such HIP device");
    c->device = hip_device;
    TD_HIP(hipSetDevice(hip_device));
    TD_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    TD_HIP(hipEventCreateWithFlags(&c->done, hipEventDisableTiming));
    TD_HIP(hipEventCreateWithFlags(&c->xev, hipEventDisableTiming));
    TD_HIP(hipEventCreateWithFlags(&c->uev, hipEventDisableTiming));
    init_decode_scratch(hip_device);
  });
  if (s != TD_OK) {
    td_destroy(c);
    return s;
  }
  *out = c;
  return TD_OK;
}

void td_destroy(td_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (td_ctx* ch : c->children) ch->parent = nullptr;
  for (td_ctx* st : c->judged_by) {
    st->judge = nullptr;
    if (st->model) st->model->set_judge(nullptr, 0.f, nullptr);
  }
  if (c->judge) {
    auto& v = c->judge->judged_by;
    v.erase(std::remove(v.begin(), v.end(), c), v.end());
    (void)hipStreamSynchronize(c->judge->stream);
  }
  if (c->d_fallbacks) (void)hipFree(c->d_fallbacks);
  if (c->parent) {
    auto& v = c->parent->children;
    v.erase(std::remove(v.begin(), v.end(), c), v.end());
    (void)hipStreamSynchronize(c->parent->stream);   // it may still write our buffers
  }
  c->map.clear();
  c->lru.clear();
  c->pool.release();
  c->model.reset();
  c->arena.release();
  c->prof.reset();
  for (float* p : {c->canvas, c->tmp, c->dec, c->outbuf, c->cond, c->gath, c->fb})
    if (p) (void)hipFree(p);
  if (c->done) (void)hipEventDestroy(c->done);
  if (c->xev) (void)hipEventDestroy(c->xev);
  if (c->uev) (void)hipEventDestroy(c->uev);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

td_status td_load_weights(td_ctx* c, const char* path) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    TD_CHECK(path, TD_E_INVAL, "null path");
    TD_HIP(hipSetDevice(c->device));
    TD_HIP(hipStreamSynchronize(c->stream));
    // the new model is built first: a file that fails to load leaves the
    // current model and its cache as they were
    std::unique_ptr<Model> m(new Model());
    m->load(path, c->stream);
    c->map.clear();
    c->lru.clear();
    c->pool.release();
    c->model.reset();
    c->pool.configure((size_t)m->d.H * m->d.H * m->d.C);
    c->model = std::move(m);
    c->stats = td_cache_stats_t{};
    c->stats.bytes_budget = c->budget;
    c->gen++;
    c->parent_gen = 0;
  });
}

td_status td_set_conditioning(td_ctx* child, td_ctx* parent) {
  if (!child) return TD_E_INVAL;
  return guarded(child, [&] {
    TD_CHECK(parent != child, TD_E_INVAL, "a model cannot condition itself");
    for (td_ctx* a = parent; a; a = a->parent)
      TD_CHECK(a != child, TD_E_INVAL, "conditioning would form a cycle");
    TD_CHECK(!parent || parent->device == child->device, TD_E_INVAL, "parent and child must share a device");
    TD_HIP(hipSetDevice(child->device));
    TD_HIP(hipStreamSynchronize(child->stream));
    child->pending = false;
    if (child->parent) {
      auto& v = child->parent->children;
      v.erase(std::remove(v.begin(), v.end(), child), v.end());
    }
    child->parent = parent;
    if (parent) parent->children.push_back(child);
    drop_cache(child);
    child->parent_gen = 0;
  });
}

td_status td_set_judge(td_ctx* student, td_ctx* teacher, float threshold) {
  if (!student) return TD_E_INVAL;
  return guarded(student, [&] {
    need_model(student);
    TD_CHECK(student->model->d.consistency, TD_E_INVAL, "a judge applies to consistency sampling only");
    TD_CHECK(teacher != student, TD_E_INVAL, "a model cannot judge itself");
    TD_CHECK(!teacher || teacher->device == student->device, TD_E_INVAL, "judge and student must share a device");
    TD_CHECK(threshold >= 0.f, TD_E_INVAL, "threshold must be >= 0");
    if (teacher) {
      TD_CHECK(teacher->model, TD_E_STATE, "the judge context has no weights");
      const ModelDesc& d = student->model->d;
      const ModelDesc& t = teacher->model->d;
      TD_CHECK(t.C == d.C && t.H == d.H && t.S == d.S && t.O == d.O, TD_E_INVAL,
               "judge and student must share channels and window layout");
    }
    TD_HIP(hipSetDevice(student->device));
    TD_HIP(hipStreamSynchronize(student->stream));
    student->pending = false;
    if (student->judge) {
      auto& v = student->judge->judged_by;
      v.erase(std::remove(v.begin(), v.end(), student), v.end());
    }
    student->judge = teacher;
    student->judge_thr = threshold;
    student->judge_gen = 0;
    if (teacher) {
      teacher->judged_by.push_back(student);
      if (!student->d_fallbacks) {
        TD_HIP(hipMalloc(&student->d_fallbacks, sizeof(unsigned long long)));
        TD_HIP(hipMemset(student->d_fallbacks, 0, sizeof(unsigned long long)));
        student->fallbacks_base = 0;
      }
    }
    drop_cache(student);
    check_judge(student, true);
  });
}

td_status td_sample_region_async(td_ctx* c, uint64_t seed, int64_t x0, int64_t y0, int32_t w, int32_t h,
                                 int32_t level, float* dev_out, size_t out_len, void* hip_stream) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    TD_CHECK(dev_out, TD_E_INVAL, "null output");
    TD_HIP(hipSetDevice(c->device));
    hipStream_t user = hip_stream == TD_STREAM_DEFAULT ? nullptr : (hipStream_t)hip_stream;
    if (hip_stream && user != c->stream) {
      // order after the caller's stream, run on ours, then make theirs wait
      // (a wait takes the event's state at the time of the call, so one
      // event serves both directions)
      TD_HIP(hipEventRecord(c->uev, user));
      TD_HIP(hipStreamWaitEvent(c->stream, c->uev, 0));
      sample_any(c, seed, x0, y0, w, h, level, dev_out, out_len);
      TD_HIP(hipEventRecord(c->uev, c->stream));
      TD_HIP(hipStreamWaitEvent(user, c->uev, 0));
    } else {
      sample_any(c, seed, x0, y0, w, h, level, dev_out, out_len);
    }
  });
}

td_status td_sample_region(td_ctx* c, uint64_t seed, int64_t x0, int64_t y0, int32_t w, int32_t h, int32_t level,
                           float* out, size_t out_len) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    TD_CHECK(out, TD_E_INVAL, "null output");
    need_model(c);
    TD_HIP(hipSetDevice(c->device));
    size_t n = level == TD_LEVEL_HEIGHT ? (size_t)std::max(w, 0) * std::max(h, 0)
                                        : (size_t)std::max(w, 0) * std::max(h, 0) * c->model->d.C;
    TD_CHECK(out_len >= n, TD_E_INVAL, "output buffer too small");
    grow(c->outbuf, c->outbuf_cap, std::max<size_t>(n, 1));
    sample_any(c, seed, x0, y0, w, h, level, c->outbuf, n);
    TD_HIP(hipMemcpyAsync(out, c->outbuf, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    TD_HIP(hipStreamSynchronize(c->stream));
    c->pending = false;
  });
}

td_status td_cache_set_budget(td_ctx* c, size_t bytes) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    c->budget = bytes;
    c->stats.bytes_budget = bytes;
    if (c->model) evict_to_budget(c);
  });
}

td_status td_cache_clear(td_ctx* c) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    TD_HIP(hipSetDevice(c->device));
    TD_HIP(hipStreamSynchronize(c->stream));
    c->pending = false;
    for (auto& kv : c->map) c->pool.give(kv.second.slot);
    c->map.clear();
    c->lru.clear();
    c->stats = td_cache_stats_t{};
    c->stats.bytes_budget = c->budget;
    c->fallbacks_base = read_fallbacks(c);
  });
}

td_status td_cache_stats(td_ctx* c, td_cache_stats_t* out) {
  if (!c || !out) return TD_E_INVAL;
  return guarded(c, [&] {
    c->stats.bytes_used = c->model ? c->map.size() * c->pool.slot_bytes() : 0;
    c->stats.bytes_budget = c->budget;
    c->stats.judge_fallbacks = read_fallbacks(c) - c->fallbacks_base;
    *out = c->stats;
  });
}

td_status td_cache_peek(td_ctx* c, uint64_t seed, int32_t level, int64_t ix, int64_t iy, float* out,
                        size_t out_len) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    need_model(c);
    TD_CHECK(out, TD_E_INVAL, "null output");
    const ModelDesc& d = c->model->d;
    size_t n = (size_t)d.H * d.H * d.C;
    TD_CHECK(out_len >= n, TD_E_INVAL, "output buffer too small");
    auto m = c->map.find(Key{seed, level, ix, iy});
    TD_CHECK(m != c->map.end(), TD_E_INVAL, "window not cached");
    TD_HIP(hipSetDevice(c->device));
    TD_HIP(hipMemcpyAsync(out, c->pool.ptr(m->second.slot), n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    TD_HIP(hipStreamSynchronize(c->stream));
  });
}

td_status td_set_option(td_ctx* c, const char* key, int64_t value) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    TD_CHECK(key, TD_E_INVAL, "null option key");
    std::string k(key);
    if (k == "batch") {
      TD_CHECK(value >= 1 && value <= (1 << 20), TD_E_INVAL, "batch must be in [1, 2^20]");
      c->batch = (int)value;
    } else if (k == "precision") {
      need_model(c);
      TD_HIP(hipStreamSynchronize(c->stream));
      c->model->set_precision((int)value);
      // cached contributions were computed at the previous precision, and
      // so were the latents of any child this model conditions
      drop_cache(c);
      c->gen++;
    } else if (k == "timing") {
      if (value && !c->prof) c->prof.reset(new Profiler());
      if (!value && c->prof) {
        TD_HIP(hipStreamSynchronize(c->stream));
        c->prof.reset();
      }
    } else if (k == "cache_budget") {
      TD_CHECK(value >= 0, TD_E_INVAL, "budget must be >= 0");
      c->budget = (size_t)value;
      if (c->model) evict_to_budget(c);
    } else {
      throw Error{TD_E_INVAL, "unknown option: " + k};
    }
  });
}

td_status td_get_info(td_ctx* c, const char* key, int64_t* value) {
  if (!c || !value) return TD_E_INVAL;
  return guarded(c, [&] {
    need_model(c);
    TD_CHECK(key, TD_E_INVAL, "null key");
    const ModelDesc& d = c->model->d;
    std::string k(key);
    if (k == "channels") *value = d.C;
    else if (k == "steps") *value = d.K;
    else if (k == "levels") *value = d.T;
    else if (k == "window") *value = d.H;
    else if (k == "stride") *value = d.S;
    else if (k == "offset") *value = d.O;
    else if (k == "factor") *value = d.factor;
    else if (k == "params") *value = (int64_t)d.params;
    else if (k == "batch") *value = auto_batch(c);
    else if (k == "precision") *value = c->model->precision();
    else if (k == "cond_channels") *value = d.Cc;
    else if (k == "cond_factor") *value = d.cond_factor;
    else if (k == "noise_step") *value = d.noise_step;
    else throw Error{TD_E_INVAL, "unknown info key: " + k};
  });
}

td_status td_denoise_windows(td_ctx* c, const float* x_dev, const float* cond_dev, int32_t n, int32_t k,
                             float* out_dev) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    need_model(c);
    const ModelDesc& d = c->model->d;
    TD_CHECK(x_dev && out_dev && n >= 0, TD_E_INVAL, "bad arguments");
    TD_CHECK(!d.Cc == !cond_dev, TD_E_INVAL, "conditioning windows are required by (and only by) a conditioned model");
    TD_CHECK(k >= 0 && k < d.K, TD_E_INVAL, "sigma index out of range");
    TD_HIP(hipSetDevice(c->device));
    if (c->pending) {
      TD_HIP(hipEventSynchronize(c->done));
      c->pending = false;
    }
    c->arena.reset();
    int maxb = auto_batch(c);
    c->model->ensure_workspace(maxb);
    c->arena.ensure((size_t)(n / maxb + 1) * (256 + (size_t)std::min(n, maxb) * 2 * sizeof(int)));
    for (int b0 = 0; b0 < n; b0 += maxb) {
      int nb = std::min(maxb, n - b0);
      auto o = c->arena.reserve((size_t)nb * 2 * sizeof(int));
      int* ho = (int*)o.first;
      for (int j = 0; j < nb; ++j) {
        ho[2 * j] = 0;
        ho[2 * j + 1] = j * d.H;
      }
      TD_HIP(hipMemcpyAsync(o.second, o.first, (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, c->stream));
      WindowBatch wb;
      wb.canvas = x_dev + (size_t)b0 * d.H * d.H * d.C;
      wb.canvas_w = d.H;
      wb.d_origins = (const int*)o.second;
      wb.d_widx = (const int*)o.second;  // analytic kind: window index (0, j*H) is unused by the UNet
      wb.n = nb;
      wb.mode = 1;
      wb.dout = out_dev + (size_t)b0 * d.H * d.H * d.C;
      if (cond_dev) wb.cond = cond_dev + (size_t)b0 * d.H * d.H * d.Cc;
      c->model->run_batch(c->stream, wb, k);
    }
    TD_HIP(hipStreamSynchronize(c->stream));
  });
}

td_status td_denoise_steps(td_ctx* c, const float* x_dev, int32_t n, int32_t k0, int32_t k1, float* out_dev) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    need_model(c);
    const ModelDesc& d = c->model->d;
    TD_CHECK(x_dev && out_dev && n >= 0, TD_E_INVAL, "bad arguments");
    TD_CHECK(!d.consistency, TD_E_INVAL, "window-local steps need an Euler (EDM) sampler");
    TD_CHECK(!d.Cc, TD_E_INVAL, "window-local steps of a conditioned model are not supported");
    TD_CHECK(0 <= k0 && k0 < k1 && k1 <= d.K, TD_E_INVAL, "steps must satisfy 0 <= k0 < k1 <= K");
    TD_HIP(hipSetDevice(c->device));
    if (c->pending) {
      TD_HIP(hipEventSynchronize(c->done));
      c->pending = false;
    }
    c->arena.reset();
    const int maxb = auto_batch(c);
    c->model->ensure_workspace(maxb);
    const size_t per = (size_t)d.H * d.H * d.C;
    c->arena.ensure((size_t)(n / maxb + 1) * (256 + (size_t)std::min(n, maxb) * 2 * sizeof(int)));
    for (int b0 = 0; b0 < n; b0 += maxb) {
      const int nb = std::min(maxb, n - b0);
      auto o = c->arena.reserve((size_t)nb * 2 * sizeof(int));
      int* ho = (int*)o.first;
      for (int j = 0; j < nb; ++j) {
        ho[2 * j] = 0;
        ho[2 * j + 1] = j * d.H;
      }
      TD_HIP(hipMemcpyAsync(o.second, o.first, (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, c->stream));
      for (int k = k0; k < k1; ++k) {
        WindowBatch wb;
        wb.canvas = (k == k0 ? x_dev : out_dev) + (size_t)b0 * per;   // Phi may overwrite its own input
        wb.canvas_w = d.H;
        wb.d_origins = (const int*)o.second;
        wb.d_widx = (const int*)o.second;
        wb.n = nb;
        wb.mode = 2;
        wb.dout = out_dev + (size_t)b0 * per;
        c->model->run_batch(c->stream, wb, k);
      }
    }
    TD_HIP(hipStreamSynchronize(c->stream));
  });
}

td_status td_noise_region(uint64_t seed, int64_t x0, int64_t y0, int32_t w, int32_t h, int32_t channels,
                          uint32_t step, float scale, int32_t accumulate, float* dev_out, void* hip_stream) {
  if (!dev_out || w < 1 || h < 1 || channels < 1 || (int64_t)w * h > (1LL << 30) ||
      (accumulate != 0 && accumulate != 1))
    return TD_E_INVAL;
  try {
    launch_noise(hip_stream == TD_STREAM_DEFAULT ? nullptr : (hipStream_t)hip_stream, seed, x0, y0, w, h, channels,
                 step, scale, 0, dev_out, accumulate);
  } catch (const Error& e) {
    return (td_status)e.status;
  }
  return TD_OK;
}

td_status td_lap_decode(td_ctx* c, const float* latent_dev, int64_t lx0, int64_t ly0, int32_t lw, int32_t lh,
                        int64_t X0, int64_t Y0, int32_t W, int32_t H, float* out_dev, void* hip_stream) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    need_model(c);
    TD_CHECK(latent_dev && out_dev && lw > 0 && lh > 0, TD_E_INVAL, "bad arguments");
    check_region(X0, Y0, W, H);
    TD_HIP(hipSetDevice(c->device));
    hipStream_t st = !hip_stream ? c->stream : hip_stream == TD_STREAM_DEFAULT ? nullptr : (hipStream_t)hip_stream;
    if (c->pending) {
      TD_HIP(hipEventSynchronize(c->done));
      c->pending = false;
    }
    Region need = decode_apron(c->model->d, Region{X0, Y0, W, H});
    TD_CHECK(need.x0 >= lx0 && need.y0 >= ly0 && need.x0 + need.w <= lx0 + lw && need.y0 + need.h <= ly0 + lh,
             TD_E_INVAL, "latent does not cover the 17-pixel decode apron");
    decode_into(c, latent_dev, Region{lx0, ly0, lw, lh}, Region{X0, Y0, W, H}, out_dev, st);
  });
}

td_status td_lap_decode_noalloc(td_ctx* c, const float* latent_dev, int64_t lx0, int64_t ly0, int32_t lw,
                                int32_t lh, int64_t X0, int64_t Y0, int32_t W, int32_t H, float* out_dev,
                                void* hip_stream) {
  if (!c) return TD_E_INVAL;
  return guarded(c, [&] {
    g_prof = nullptr;   // per-launch timing would create events
    need_model(c);
    TD_CHECK(latent_dev && out_dev && lw > 0 && lh > 0, TD_E_INVAL, "bad arguments");
    check_region(X0, Y0, W, H);
    TD_HIP(hipSetDevice(c->device));
    hipStream_t st = !hip_stream ? c->stream : hip_stream == TD_STREAM_DEFAULT ? nullptr : (hipStream_t)hip_stream;
    if (c->pending) {
      TD_HIP(hipEventSynchronize(c->done));
      c->pending = false;
    }
    Region need = decode_apron(c->model->d, Region{X0, Y0, W, H});
    TD_CHECK(need.x0 >= lx0 && need.y0 >= ly0 && need.x0 + need.w <= lx0 + lw && need.y0 + need.h <= ly0 + lh,
             TD_E_INVAL, "latent does not cover the 17-pixel decode apron");
    DecodeArgs a = decode_args(c, latent_dev, Region{lx0, ly0, lw, lh}, Region{X0, Y0, W, H}, out_dev);
    const size_t wf = decode_work_floats(a);
    TD_CHECK(2 * wf <= kDecodeScratchFloats, TD_E_INVAL,
             "region too large for the fixed decode scratch: needs 2 x " + std::to_string(wf) + " floats, has " +
                 std::to_string(kDecodeScratchFloats));
    float* scratch = decode_scratch(c->device);
    TD_CHECK(scratch, TD_E_STATE, "decode scratch not set up on this device");
    a.work0 = scratch;   // both fully written by the decode before they are read
    a.work1 = scratch + wf;
    launch_decode(st, a);
  });
}

td_status td_lap_encode(td_ctx* c, const float* height_dev, int64_t X0, int64_t Y0, int32_t W, int32_t H,
                        float* latent_dev, size_t latent_len, int64_t geom[4], void* hip_stream) {
  if (!c || !geom) return TD_E_INVAL;
  return guarded(c, [&] {
    need_model(c);
    const ModelDesc& d = c->model->d;
    TD_CHECK(d.factor == 8, TD_E_STATE, "encode: the decode factor must be 8");
    TD_CHECK(W >= 1 && H >= 1 && W % 8 == 0 && H % 8 == 0 && floordiv64(X0, 8) * 8 == X0 &&
                 floordiv64(Y0, 8) * 8 == Y0, TD_E_INVAL, "encode: the region must be 8-aligned");
    check_region(X0, Y0, W, H);
    const int R = d.blur_radius;
    const int64_t ow = W / 8 - 2 * R - 2, oh = H / 8 - 2 * R - 2;
    TD_CHECK(ow >= 1 && oh >= 1, TD_E_INVAL, "encode: region too small for the blur and up8 aprons");
    geom[0] = X0 / 8 + R + 1;
    geom[1] = Y0 / 8 + R + 1;
    geom[2] = ow;
    geom[3] = oh;
    if (!latent_dev) return;
    TD_CHECK(height_dev, TD_E_INVAL, "encode: null height");
    TD_CHECK(latent_len >= (size_t)(ow * oh * d.C), TD_E_INVAL, "encode: latent buffer too small");
    TD_HIP(hipSetDevice(c->device));
    hipStream_t st = !hip_stream ? c->stream : hip_stream == TD_STREAM_DEFAULT ? nullptr : (hipStream_t)hip_stream;
    if (c->pending) {
      TD_HIP(hipEventSynchronize(c->done));
      c->pending = false;
    }
    const size_t nb = (size_t)(W / 8) * (H / 8);
    grow(c->dec, c->dec_cap, 2 * nb);
    EncodeArgs a{};
    a.height = height_dev;
    a.W = W;
    a.H = H;
    a.C = d.C;
    a.sigma_low = (float)d.sigma_low;
    a.sigma_res = (float)d.sigma_res;
    a.taps = c->model->decode_taps();
    a.radius = R;
    a.atoms = c->model->decode_atoms();
    a.work0 = c->dec;
    a.work1 = c->dec + nb;
    a.latent = latent_dev;
    launch_encode(st, a);
  });
}

td_status td_kappa(int64_t x0, int64_t y0, int64_t w, int64_t h, int32_t size, int32_t stride, int32_t offset,
                   int64_t out[4]) {
  if (!out || size < 1 || stride < 1 || w < 1 || h < 1) return TD_E_INVAL;
  Kappa k = kappa(Region{x0, y0, w, h}, size, stride, offset);
  out[0] = k.ix0;
  out[1] = k.ix1;
  out[2] = k.iy0;
  out[3] = k.iy1;
  return k.empty ? TD_E_INVAL : TD_OK;
}

td_status td_cone_windows(int64_t x0, int64_t y0, int64_t w, int64_t h, int32_t level, int32_t steps, int32_t size,
                          int32_t stride, int32_t offset, uint64_t* count) {
  if (!count || size < 1 || stride < 1 || w < 1 || h < 1 || level < 0 || level > steps) return TD_E_INVAL;
  uint64_t n = 0;
  Region R{x0, y0, w, h};
  for (int t = level; t < steps; ++t) {
    Kappa k = kappa(R, size, stride, offset);
    if (k.empty) break;
    n += (uint64_t)k.count();
    R = Region{k.ix0 * stride + offset, k.iy0 * stride + offset, (k.ix1 - k.ix0) * stride + size,
               (k.iy1 - k.iy0) * stride + size};
  }
  *count = n;
  return TD_OK;
}

td_status td_kernel_stats(td_ctx* c, td_kernel_stat_t* out, int32_t cap, int32_t* count, int32_t reset) {
  if (!c || !count || cap < 0 || (cap > 0 && !out)) return TD_E_INVAL;
  return guarded(c, [&] {
    TD_CHECK(c->prof, TD_E_STATE, "timing is off (td_set_option \"timing\" 1)");
    TD_HIP(hipSetDevice(c->device));
    c->prof->resolve();
    int n = 0;
    for (int k = 0; k < K_NCLASS; ++k) {
      const Profiler::Total& t = c->prof->tot[k];
      if (!t.launches) continue;
      if (n < cap) {
        td_kernel_stat_t& o = out[n];
        std::memset(&o, 0, sizeof(o));
        std::strncpy(o.name, kclass_name(k), sizeof(o.name) - 1);
        o.launches = t.launches;
        o.ms = t.ms;
        o.flops = t.flops;
        o.bytes = t.bytes;
      }
      ++n;
    }
    *count = n;
    if (reset) c->prof->reset();
  });
}

const char* td_last_error(const td_ctx* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"

// ====================================================================== serving
//
// Continuous batching of region queries.  A query is planned when admitted
// (HBM budget, in-flight limit): its cone's windows are looked up in the
// cache; windows another in-flight query is already going to evaluate are
// shared, the rest become tasks owned by this query.  Every scheduling round
// (td_server_progress) builds the level canvases whose inputs have been
// enqueued, then runs ONE batched denoiser round over ready tasks of one
// level, drawn from any number of queries (the window gather copies each
// task's input out of its owner's canvas), so queries admitted while others
// are in flight share the GPU with them.  Everything runs on the context's
// stream in enqueue order, which is the only synchronisation the data needs;
// the host tracks completion with one event per query.  Results equal the
// same queries run alone, bit for bit: every window is evaluated with the
// same batch-invariant kernels and blended in canonical order.

namespace td {
namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SrvTask {
  Key key;
  uint32_t slot;
  uint64_t q;       // owning query (its canvas holds the input)
  int li;           // owning level index
  int ox, oy;       // window origin relative to the owner's canvas
  bool enq = false;
};

struct SrvLevel {
  Level L;                 // t, region, kappa, in_region (fresh = owned windows)
  std::vector<int> own;    // owned task ids
  float* canvas = nullptr;
  size_t canvas_n = 0;
  bool built = false;
  size_t n_enq = 0;
};

struct SrvQuery {
  uint64_t ticket = 0;
  td_request r{};
  double t_sub = 0, t_done = 0;
  int state = 0;           // 0 queued, 1 active, 2 result enqueued, 3 done
  std::vector<SrvLevel> lv;
  int cur = -1;
  hipEvent_t ev = nullptr;
  size_t mem = 0;
  // conditioned model: the parent latent under this query's new windows,
  // written on the parent's stream; cond_ev marks its completion, which the
  // child's stream waits for before its first batch with this query's windows
  float* cond = nullptr;
  Region cond_r{};
  hipEvent_t cond_ev = nullptr;
  bool cond_pending = false;
};

constexpr int kRing = 8;

}  // namespace
}  // namespace td

struct td_server {
  td_ctx* c = nullptr;
  size_t budget = 0;
  int max_inflight = 1;
  int maxb = 1;
  uint64_t next_ticket = 1;
  std::deque<uint64_t> queued;
  std::vector<uint64_t> active;
  std::unordered_map<uint64_t, td::SrvQuery> q;
  std::vector<td::SrvTask> tasks;   // slab indexed by task id; ids are reused
  std::vector<int> free_tasks;
  std::unordered_map<td::Key, int, td::KeyHash> pending;   // not yet enqueued
  std::map<int, std::deque<int>> ready;                    // level -> ready task ids (FIFO)
  size_t mem_used = 0;
  td::Arena ring[td::kRing];
  hipEvent_t ring_ev[td::kRing] = {};
  bool ring_used[td::kRing] = {};
  hipEvent_t ring_pev[td::kRing] = {};   // the parent's work that used the slot's arena
  bool ring_pused[td::kRing] = {};
  bool parent_round = false;             // parent work issued in the current round
  // queries admitted in this round whose parent latent is still to be
  // sampled (one batched parent call per round)
  std::vector<uint64_t> parent_wait;
  uint64_t round = 0;
  bool failed = false;   // a round threw part-way: in-flight state is not trusted
  float* batch_in = nullptr;
  size_t batch_cap = 0;
  std::multimap<size_t, float*> free_canvas;   // capacity -> free canvas
  std::vector<float*> all_canvas;
  std::unordered_map<float*, size_t> canvas_cap;
  td_server_stats_t stats{};
};

namespace td {
namespace {

float* take_canvas(td_server* s, size_t n) {
  auto it = s->free_canvas.lower_bound(n);
  if (it != s->free_canvas.end() && it->first <= 2 * n + (1 << 20)) {
    float* p = it->second;
    s->free_canvas.erase(it);
    return p;
  }
  size_t cap = std::max<size_t>(n, 1 << 18);
  float* p = nullptr;
  TD_HIP(hipMalloc(&p, cap * sizeof(float)));
  s->all_canvas.push_back(p);
  s->canvas_cap[p] = cap;
  s->stats.canvas_bytes += cap * sizeof(float);
  return p;
}

void give_canvas(td_server* s, float* p) {
  if (p) s->free_canvas.emplace(s->canvas_cap[p], p);
}

// Upper bound of the device bytes a query needs while in flight.
size_t query_bytes(td_ctx* c, const td_request& r) {
  const ModelDesc& d = c->model->d;
  size_t slot = c->pool.slot_bytes();
  size_t bytes = 0;
  Region R{r.x0, r.y0, r.w, r.h};
  for (int t = r.level; t < d.T; ++t) {
    Kappa k = kappa(R, d.H, d.S, d.O);
    if (k.empty) break;
    bytes += (size_t)k.count() * slot;
    R = Region{k.ix0 * d.S + d.O, k.iy0 * d.S + d.O, (k.ix1 - k.ix0) * d.S + d.H, (k.iy1 - k.iy0) * d.S + d.H};
    bytes += (size_t)R.w * R.h * d.C * sizeof(float);
  }
  if (d.Cc) {   // the parent latent under the cone
    const Region pr = parent_region(d, R);
    bytes += (size_t)pr.w * pr.h * d.Cc * sizeof(float);
  }
  return bytes;
}

void plan_query(td_server* s, SrvQuery& Q, Arena& arena) {
  td_ctx* c = s->c;
  const ModelDesc& d = c->model->d;
  check_parent(c, s->active.empty());
  Region R{Q.r.x0, Q.r.y0, Q.r.w, Q.r.h};
  for (int t = Q.r.level; t < d.T; ++t) {
    SrvLevel S;
    S.L.t = t;
    S.L.region = R;
    S.L.k = kappa(R, d.H, d.S, d.O);
    if (!S.L.k.empty) {
      int64_t mnx = INT64_MAX, mxx = INT64_MIN, mny = INT64_MAX, mxy = INT64_MIN;
      for (int64_t iy = S.L.k.iy0; iy <= S.L.k.iy1; ++iy)
        for (int64_t ix = S.L.k.ix0; ix <= S.L.k.ix1; ++ix) {
          Key key{Q.r.seed, t, ix, iy};
          auto ins = c->map.try_emplace(key);
          if (!ins.second) {
            ins.first->second.pins++;
            touch(c, ins.first->second, key);
            c->stats.hits++;
            continue;
          }
          int id;
          if (!s->free_tasks.empty()) {
            id = s->free_tasks.back();
            s->free_tasks.pop_back();
          } else {
            id = (int)s->tasks.size();
            s->tasks.emplace_back();
          }
          SrvTask& T = s->tasks[id];
          T = SrvTask{};
          T.key = key;
          T.slot = c->pool.take();
          T.q = Q.ticket;
          T.li = (int)Q.lv.size();
          c->lru.push_front(key);
          ins.first->second = Entry{T.slot, 1, c->lru.begin()};
          s->pending[key] = id;
          S.own.push_back(id);
          S.L.fresh.push_back({ix, iy});
          mnx = std::min(mnx, ix);
          mxx = std::max(mxx, ix);
          mny = std::min(mny, iy);
          mxy = std::max(mxy, iy);
        }
      if (!S.own.empty()) {
        S.L.in_region = Region{mnx * d.S + d.O, mny * d.S + d.O, (mxx - mnx) * d.S + d.H, (mxy - mny) * d.S + d.H};
        for (int id : S.own) {
          SrvTask& T = s->tasks[id];
          T.ox = (int)(T.key.ix * d.S + d.O - S.L.in_region.x0);
          T.oy = (int)(T.key.iy * d.S + d.O - S.L.in_region.y0);
        }
        c->stats.misses += S.own.size();
        c->stats.denoiser_evals += (uint64_t)S.own.size() * c->model->level_steps(t);
        if (t < 64) c->stats.windows_evaluated[t] += S.own.size();
      }
    }
    Q.lv.push_back(std::move(S));
    const SrvLevel& B = Q.lv.back();
    if (B.L.k.empty || B.own.empty()) break;
    R = B.L.in_region;
  }
  Q.cur = (int)Q.lv.size() - 1;
  if (d.Cc) {
    Region hull{0, 0, 0, 0};
    for (const SrvLevel& S : Q.lv)
      if (!S.own.empty()) hull = region_union(hull, S.L.in_region);
    if (hull.w > 0) {
      const Region pr = parent_region(d, hull);
      Q.cond = take_canvas(s, (size_t)pr.w * pr.h * d.Cc);
      if (!Q.cond_ev) TD_HIP(hipEventCreateWithFlags(&Q.cond_ev, hipEventDisableTiming));
      if (c->parent->model->d.Cc == 0) {   // batched with the round's other admissions
        Q.cond_r = hull;                   // (child pixels until the parent call)
        s->parent_wait.push_back(Q.ticket);
      } else {
        sample_parent(c, arena, Q.r.seed, hull, Q.cond, &Q.cond_r, Q.cond_ev);
        Q.cond_pending = true;
        s->parent_round = true;
      }
    }
  }
}

bool all_enqueued(td_server* s, uint64_t seed, const Level& L) {
  if (L.k.empty) return true;
  for (int64_t iy = L.k.iy0; iy <= L.k.iy1; ++iy)
    for (int64_t ix = L.k.ix0; ix <= L.k.ix1; ++ix)
      if (s->pending.count(Key{seed, L.t, ix, iy})) return false;
  return true;
}

// Advance one query as far as the enqueued work allows.
void advance(td_server* s, SrvQuery& Q, Arena& arena) {
  td_ctx* c = s->c;
  const ModelDesc& d = c->model->d;
  hipStream_t st = c->stream;
  while (Q.state == 1) {
    if (Q.cur >= 0) {
      SrvLevel& S = Q.lv[Q.cur];
      if (S.own.empty()) {
        Q.cur--;
        continue;
      }
      if (!S.built) {
        const int tn = S.L.t + 1;
        const bool below = Q.cur + 1 < (int)Q.lv.size();
        if (tn != d.T && below && !all_enqueued(s, Q.r.seed, Q.lv[Q.cur + 1].L)) return;
        const Region& cr = S.L.in_region;
        S.canvas_n = (size_t)cr.w * cr.h * d.C;
        S.canvas = take_canvas(s, S.canvas_n);
        if (tn == d.T) {
          launch_noise(st, Q.r.seed, cr.x0, cr.y0, (int)cr.w, (int)cr.h, d.C, 0, (float)d.sched[0], 0, S.canvas);
        } else if (!below || Q.lv[Q.cur + 1].L.k.empty) {
          launch_fill(st, S.canvas, S.canvas_n, 0.f);
        } else {
          blend_into(c, arena, Q.r.seed, Q.lv[Q.cur + 1].L, cr, 0, S.canvas);
          unpin_level(c, Q.r.seed, Q.lv[Q.cur + 1].L);
        }
        S.built = true;
        for (int id : S.own) s->ready[S.L.t].push_back(id);
      }
      if (S.n_enq < S.own.size()) return;
      give_canvas(s, S.canvas);       // later users are stream-ordered after its readers
      S.canvas = nullptr;
      Q.cur--;
      continue;
    }
    // every own window enqueued: its conditioning has been gathered
    if (Q.cond) {
      give_canvas(s, Q.cond);
      Q.cond = nullptr;
    }
    // every level evaluated: the result is the blend of the query level
    const Level& top = Q.lv[0].L;
    if (!all_enqueued(s, Q.r.seed, top)) return;
    const size_t n = (size_t)Q.r.w * Q.r.h * d.C;
    if (top.k.empty) {
      launch_fill(st, Q.r.dev_out, n, 0.f);
    } else {
      blend_into(c, arena, Q.r.seed, top, Region{Q.r.x0, Q.r.y0, Q.r.w, Q.r.h}, 1, Q.r.dev_out);
      unpin_level(c, Q.r.seed, top);
    }
    TD_HIP(hipEventRecord(Q.ev, st));
    Q.state = 2;
    s->mem_used -= Q.mem;
    c->stats.queries++;
  }
}

// One batched denoiser round over ready tasks of a single level.
bool run_round_batch(td_server* s, Arena& arena) {
  td_ctx* c = s->c;
  const ModelDesc& d = c->model->d;
  hipStream_t st = c->stream;
  int best = -1;
  size_t bestn = 0;
  for (auto& kv : s->ready)
    if (kv.second.size() > bestn || (kv.second.size() == bestn && bestn && kv.first > best)) {
      best = kv.first;
      bestn = kv.second.size();
    }
  if (best < 0 || bestn == 0) return false;
  std::deque<int>& dq = s->ready[best];
  const int nb = (int)std::min<size_t>(dq.size(), (size_t)s->maxb);
  const size_t per = (size_t)d.H * d.H * d.C;
  if ((size_t)nb * per > s->batch_cap) {
    TD_HIP(hipStreamSynchronize(st));
    if (s->batch_in) TD_HIP(hipFree(s->batch_in));
    s->batch_cap = (size_t)s->maxb * per;
    TD_HIP(hipMalloc(&s->batch_in, s->batch_cap * sizeof(float)));
  }
  auto src = arena.reserve((size_t)nb * sizeof(float*));
  auto pit = arena.reserve((size_t)nb * sizeof(int));
  auto org = arena.reserve((size_t)nb * 2 * sizeof(int));
  auto wix = arena.reserve((size_t)nb * 2 * sizeof(int));
  auto slo = arena.reserve((size_t)nb * sizeof(float*));
  const float** hs = (const float**)src.first;
  int* hp = (int*)pit.first;
  int* ho = (int*)org.first;
  int* hw = (int*)wix.first;
  float** hsl = (float**)slo.first;
  std::vector<int> ids(nb);
  for (int j = 0; j < nb; ++j) {
    ids[j] = dq.front();
    dq.pop_front();
    SrvTask& T = s->tasks[ids[j]];
    SrvQuery& O = s->q[T.q];
    SrvLevel& S = O.lv[T.li];
    hs[j] = S.canvas + ((size_t)T.oy * S.L.in_region.w + T.ox) * d.C;
    hp[j] = (int)S.L.in_region.w;
    ho[2 * j] = 0;
    ho[2 * j + 1] = j * d.H;
    hw[2 * j] = (int)T.key.ix;
    hw[2 * j + 1] = (int)T.key.iy;
    hsl[j] = c->pool.ptr(T.slot);
  }
  TD_HIP(hipMemcpyAsync(src.second, src.first, (size_t)nb * sizeof(float*), hipMemcpyHostToDevice, st));
  TD_HIP(hipMemcpyAsync(pit.second, pit.first, (size_t)nb * sizeof(int), hipMemcpyHostToDevice, st));
  TD_HIP(hipMemcpyAsync(org.second, org.first, (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, st));
  TD_HIP(hipMemcpyAsync(wix.second, wix.first, (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, st));
  TD_HIP(hipMemcpyAsync(slo.second, slo.first, (size_t)nb * sizeof(float*), hipMemcpyHostToDevice, st));
  launch_gather(st, (const float* const*)src.second, (const int*)pit.second, nb, d.H, d.C, s->batch_in);
  std::vector<CondSrc> cs(d.Cc ? nb : 0);
  for (int j = 0; j < (int)cs.size(); ++j) {
    const SrvTask& T = s->tasks[ids[j]];
    SrvQuery& O = s->q[T.q];
    if (O.cond_pending) {   // the parent latent this window reads must be written
      TD_HIP(hipStreamWaitEvent(st, O.cond_ev, 0));
      O.cond_pending = false;
    }
    cs[j] = cond_src(d, O.cond, O.cond_r.w, O.cond_r.x0 * d.cond_factor, O.cond_r.y0 * d.cond_factor, T.key.ix,
                     T.key.iy);
  }
  if (d.Cc) cond_batch(c, arena, cs.data(), nb);
  std::vector<uint64_t> seeds(nb);
  for (int j = 0; j < nb; ++j) seeds[j] = s->q[s->tasks[ids[j]].q].r.seed;
  WindowBatch wb;
  wb.canvas = s->batch_in;
  wb.canvas_w = d.H;
  wb.d_origins = (const int*)org.second;
  wb.d_widx = (const int*)wix.second;
  wb.d_slots = (float* const*)slo.second;
  wb.n = nb;
  wb.mode = 0;
  wb.h_widx = hw;
  wb.h_seeds = seeds.data();
  if (d.Cc) wb.cond = c->model->cond_buffer();
  c->model->run_level(st, wb, best);
  c->stats.batches++;
  s->stats.batched_windows += nb;
  for (int id : ids) {
    SrvTask& T = s->tasks[id];
    T.enq = true;
    s->pending.erase(T.key);
    s->q[T.q].lv[T.li].n_enq++;
  }
  for (int id : ids) s->free_tasks.push_back(id);
  if (dq.empty()) s->ready.erase(best);
  return true;
}

void admit(td_server* s, Arena& arena) {
  while (!s->queued.empty() && (int)s->active.size() < s->max_inflight) {
    SrvQuery& Q = s->q[s->queued.front()];
    size_t need = query_bytes(s->c, Q.r);
    if (!s->active.empty() && s->mem_used + need > s->budget) break;
    s->queued.pop_front();
    Q.mem = need;
    s->mem_used += need;
    plan_query(s, Q, arena);
    Q.state = 1;
    s->active.push_back(Q.ticket);
    s->stats.admitted++;
  }
  if (!s->parent_wait.empty()) {
    td_ctx* c = s->c;
    std::vector<RegionJob> hulls;
    for (uint64_t t : s->parent_wait) {
      SrvQuery& Q = s->q[t];
      hulls.push_back(RegionJob{Q.r.seed, Q.cond_r, Q.cond});
    }
    std::vector<Region> rcs;
    sample_parents(c, arena, hulls, &rcs);
    for (size_t i = 0; i < s->parent_wait.size(); ++i) {
      SrvQuery& Q = s->q[s->parent_wait[i]];
      Q.cond_r = rcs[i];
      TD_HIP(hipEventRecord(Q.cond_ev, c->parent->stream));
      Q.cond_pending = true;
    }
    s->parent_wait.clear();
    s->parent_round = true;
  }
}

void server_round(td_server* s) {
  td_ctx* c = s->c;
  const int slot = (int)(s->round % kRing);
  if (s->ring_used[slot]) TD_HIP(hipEventSynchronize(s->ring_ev[slot]));
  if (s->ring_pused[slot]) TD_HIP(hipEventSynchronize(s->ring_pev[slot]));
  s->ring_pused[slot] = false;
  s->parent_round = false;
  Arena& arena = s->ring[slot];
  arena.reset();
  admit(s, arena);
  size_t need = 65536;   // metadata of this round: pointer grids + one batch
  for (uint64_t t : s->active) {
    const SrvQuery& Q = s->q[t];
    for (const SrvLevel& S : Q.lv) need += (size_t)S.L.k.count() * sizeof(float*) + 256;
  }
  need += (size_t)s->maxb * (48 + sizeof(CondSrc)) + 6 * 256;
  arena.ensure(need);
  judge_fence(c, true);
  for (uint64_t t : s->active) advance(s, s->q[t], arena);
  if (run_round_batch(s, arena)) s->stats.rounds++;
  for (uint64_t t : s->active) advance(s, s->q[t], arena);
  judge_fence(c, false);
  TD_HIP(hipEventRecord(s->ring_ev[slot], c->stream));
  s->ring_used[slot] = true;
  if (s->parent_round) {
    TD_HIP(hipEventRecord(s->ring_pev[slot], c->parent->stream));
    s->ring_pused[slot] = true;
  }
  s->round++;
  // completions
  std::vector<uint64_t> still;
  for (uint64_t t : s->active) {
    SrvQuery& Q = s->q[t];
    if (Q.state == 2) {
      hipError_t e = hipEventQuery(Q.ev);
      if (e == hipSuccess) {
        Q.state = 3;
        Q.t_done = now_ms();
        s->stats.completed++;
      } else if (e != hipErrorNotReady) {
        TD_HIP(e);
      }
      (void)hipGetLastError();   // "not ready" is a status, not an error
    }
    if (Q.state != 3) still.push_back(t);
  }
  s->active.swap(still);
  evict_to_budget(c);
}

}  // namespace
}  // namespace td

extern "C" {

td_status td_server_create(td_ctx* c, size_t hbm_budget, int32_t max_inflight, td_server** out) {
  if (!c || !out || max_inflight < 1) return TD_E_INVAL;
  *out = nullptr;
  td_server* s = nullptr;
  td_status st = guarded(c, [&] {
    need_model(c);
    TD_HIP(hipSetDevice(c->device));
    s = new td_server();
    s->c = c;
    s->budget = hbm_budget;
    s->max_inflight = max_inflight;
    s->maxb = std::min(auto_batch(c), 4096);
    c->map.reserve(std::max<size_t>(c->map.size(), (size_t)1 << 21));   // no rehash while serving
    s->pending.reserve((size_t)1 << 16);
    c->model->ensure_workspace(s->maxb);
    for (int i = 0; i < kRing; ++i) {
      TD_HIP(hipEventCreateWithFlags(&s->ring_ev[i], hipEventDisableTiming));
      TD_HIP(hipEventCreateWithFlags(&s->ring_pev[i], hipEventDisableTiming));
    }
  });
  if (st != TD_OK) {
    td_server_destroy(s);
    return st;
  }
  *out = s;
  return TD_OK;
}

void td_server_destroy(td_server* s) {
  if (!s) return;
  td_ctx* c = s->c;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->parent) (void)hipStreamSynchronize(c->parent->stream);   // parent latents still being written
  // release what unfinished queries hold: pins and not-yet-evaluated slots
  // (after a failed round, windows may have been claimed and never written:
  // the whole cache goes)
  if (s->failed) {
    drop_cache(c);
    s->pending.clear();
  }
  for (auto& kv : s->pending) {
    auto m = c->map.find(kv.first);
    if (m != c->map.end()) {
      c->pool.give(m->second.slot);
      c->lru.erase(m->second.lru);
      c->map.erase(m);
    }
  }
  for (auto& kv : s->q) {
    SrvQuery& Q = kv.second;
    if (Q.state == 1) {
      for (int i = std::max(Q.cur, 0); i < (int)Q.lv.size(); ++i) unpin_level(c, Q.r.seed, Q.lv[i].L);
    }
    if (Q.ev) (void)hipEventDestroy(Q.ev);
    if (Q.cond_ev) (void)hipEventDestroy(Q.cond_ev);
  }
  for (float* p : s->all_canvas) (void)hipFree(p);
  if (s->batch_in) (void)hipFree(s->batch_in);
  for (int i = 0; i < kRing; ++i) {
    if (s->ring_ev[i]) (void)hipEventDestroy(s->ring_ev[i]);
    if (s->ring_pev[i]) (void)hipEventDestroy(s->ring_pev[i]);
  }
  delete s;
}

td_status td_server_submit(td_server* s, const td_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return TD_E_INVAL;
  td_ctx* c = s->c;
  return guarded(c, [&] {
    need_model(c);
    const ModelDesc& d = c->model->d;
    check_region(r->x0, r->y0, r->w, r->h);
    TD_CHECK(r->level >= 0 && r->level < d.T, TD_E_INVAL, "server queries take latent levels 0..T-1");
    TD_CHECK(r->dev_out && r->out_len >= (size_t)r->w * r->h * d.C, TD_E_INVAL, "output buffer too small");
    SrvQuery Q;
    Q.ticket = s->next_ticket++;
    Q.r = *r;
    Q.t_sub = now_ms();
    TD_HIP(hipEventCreateWithFlags(&Q.ev, hipEventDisableTiming));
    const uint64_t t = Q.ticket;
    s->q[t] = std::move(Q);
    s->queued.push_back(t);
    s->stats.submitted++;
    *ticket = t;
  });
}

td_status td_server_progress(td_server* s, int32_t rounds, int32_t* in_flight) {
  if (!s || rounds < 0) return TD_E_INVAL;
  td_ctx* c = s->c;
  return guarded(c, [&] {
    TD_CHECK(!s->failed, TD_E_STATE, "an earlier round failed: destroy the server");
    TD_HIP(hipSetDevice(c->device));
    try {
      for (int i = 0; i < rounds; ++i) server_round(s);
    } catch (...) {
      s->failed = true;
      throw;
    }
    if (in_flight) *in_flight = (int32_t)(s->active.size() + s->queued.size());
  });
}

td_status td_server_poll(td_server* s, uint64_t ticket, int32_t* done, double* latency_ms) {
  if (!s || !done) return TD_E_INVAL;
  auto it = s->q.find(ticket);
  if (it == s->q.end()) return TD_E_INVAL;
  SrvQuery& Q = it->second;
  *done = Q.state == 3;
  if (Q.state == 3) {
    if (latency_ms) *latency_ms = Q.t_done - Q.t_sub;
    if (Q.ev) (void)hipEventDestroy(Q.ev);
    if (Q.cond_ev) (void)hipEventDestroy(Q.cond_ev);
    s->q.erase(it);
  }
  return TD_OK;
}

td_status td_server_stats(td_server* s, td_server_stats_t* out) {
  if (!s || !out) return TD_E_INVAL;
  s->stats.in_flight = s->active.size();
  s->stats.queued = s->queued.size();
  s->stats.mem_in_flight = s->mem_used;
  *out = s->stats;
  return TD_OK;
}

}  // extern "C"
