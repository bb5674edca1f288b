// C-ABI entry points: context, matrix handles, build, truncation, batched
// multiply and read-back helpers.  All device work goes to the kernels in the
// k_*.hip files; this file only sizes, allocates (from the caller's arena),
// enqueues and reads back.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace spamm;

struct spamm_ctx {
  Ctx c;
};

namespace spamm {

spamm_status fail(Ctx* c, spamm_status s, const std::string& msg) {
  if (c) c->last_error = msg;
  return s;
}

void* Ctx::stage(size_t bytes) {
  if (bytes <= host_stage_bytes) return host_stage;
  if (host_stage) (void)hipHostFree(host_stage);
  host_stage = nullptr;
  host_stage_bytes = 0;
  size_t want = std::max<size_t>(bytes, size_t(1) << 20);
  if (hipHostMalloc(&host_stage, want, hipHostMallocDefault) != hipSuccess) return nullptr;
  host_stage_bytes = want;
  return host_stage;
}

bool Ctx::results(size_t bytes) {
  if (bytes <= res_bytes) return true;
  if (res_host) {  // kernels of earlier calls may still write the old buffer
    if (hipStreamSynchronize(stream) != hipSuccess) return false;
    (void)hipHostFree(res_host);
  }
  res_host = res_dev = nullptr;
  res_bytes = 0;
  const size_t want = std::max<size_t>((bytes + 4095) / 4096 * 4096, size_t(1) << 20);
  void* h = nullptr;
  if (hipHostMalloc(&h, want, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return false;
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
    (void)hipHostFree(h);
    return false;
  }
  res_host = static_cast<char*>(h);
  res_dev = static_cast<char*>(d);
  res_bytes = want;
  return true;
}

hipEvent_t Ctx::get_event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipError_t Ctx::collect_timing() {
  hipError_t err = hipStreamSynchronize(stream);
  if (err != hipSuccess) return err;
  for (auto& p : pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      t_ms[p.cls] += ms;
      t_cnt[p.cls] += 1;
    }
    event_pool.push_back(p.a);
    event_pool.push_back(p.b);
  }
  pending.clear();
  return hipSuccess;
}

}  // namespace spamm

size_t spamm_mat::device_bytes() const {
  size_t b = 0;
  for (auto* r : {&slot, &norms, &rm_sqrt, &rm_slot, &cm_sqrt, &cm_slot, &ranges, &plan_off, &plan_pairs, &plan_bnd})
    if (*r) b += (*r)->bytes;
  if (store) {
    for (auto* r : {&store->keys, &store->f64, &store->f32, &store->bf16, &store->bf16t})
      if (*r) b += (*r)->bytes;
  }
  return b;
}

namespace {

constexpr int kMaxL = 11;  // G <= 2048

bool leaf_ok(int bs) { return bs == 16 || bs == 32 || bs == 64 || bs == 128 || bs == 256; }

// Whether a launch group's products run in quads of sibling C leaves:
// option 1 always, 0 never, -1: at leaf 64 when the group's C leaves
// average at least a precision's threshold of kept products (below it the
// quads' siblings share few k, a step often serves one or two children, and
// the one-leaf kernel is faster; the thresholds are the measured crossovers
// on 3D and 1D decay, FP64 / FP32 multiply-bound, BF16 forms load-bound);
// at leaves 128 and 256 (every child keeps every step) for FP64 only, where
// they measured 1.07-1.26x faster, the other precisions 0.7-1.1x.
bool quad_group(const Ctx* c, int prec, int bs, int64_t kept, int64_t leaves) {
  if (c->gemm_quad == 0 || !gemm_quad_supported(prec, bs)) return false;
  if (c->gemm_quad == 1) return true;
  if (bs > 64) return prec == SPAMM_F64;
  // measured crossovers against the one-leaf GEMM (3D and 1D decay)
  const int64_t per_leaf = prec == SPAMM_F64 ? 32 : prec == SPAMM_F32 ? 128 : 16;
  return kept >= per_leaf * std::max<int64_t>(leaves, 1);
}

void grid_of(int64_t n, int bs, int& G, int& L) {
  const int64_t g = (n + bs - 1) / bs;
  G = 1;
  L = 0;
  while (G < g) {
    G *= 2;
    ++L;
  }
}

template <typename T>
T* P(const RegionP& r) {
  return r ? static_cast<T*>(r->ptr()) : nullptr;
}

struct Sync {
  Ctx* c;
  hipEvent_t ev = nullptr;
};

spamm_status sync_stream(Ctx* c) {
  SPAMM_HIP(c, hipStreamSynchronize(c->stream));
  return SPAMM_OK;
}

spamm_status upload(Ctx* c, void* dev, const void* host, size_t bytes) {
  if (bytes == 0) return SPAMM_OK;
  const size_t need = (bytes + 255) / 256 * 256;
  if (need > c->up_bytes) {  // (re)allocate the ring once every copy out of it is done
    SPAMM_HIP(c, hipStreamSynchronize(c->stream));
    for (auto& r : c->up_inflight) c->up_events.push_back(r.ev);
    c->up_inflight.clear();
    if (c->up_ring) SPAMM_HIP(c, hipHostFree(c->up_ring));
    c->up_ring = nullptr;
    c->up_bytes = 0;
    const size_t want = std::max<size_t>(need, size_t(8) << 20);
    void* p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess)
      return fail(c, SPAMM_EDEVICE, "hipHostMalloc of the upload ring failed");
    c->up_ring = static_cast<char*>(p);
    c->up_bytes = want;
    c->up_head = 0;
  }
  if (c->up_head + need > c->up_bytes) c->up_head = 0;
  const size_t s = c->up_head, e = s + need;
  // wait for the newest earlier copy that read any of [s, e); events on one
  // stream complete in order, so every copy before it is done too
  int last = -1;
  for (int i = 0; i < int(c->up_inflight.size()); ++i) {
    const auto& r = c->up_inflight[i];
    if (r.s < e && s < r.e) last = i;
  }
  if (last >= 0) SPAMM_HIP(c, hipEventSynchronize(c->up_inflight[last].ev));
  for (int i = 0; i <= last; ++i) {
    c->up_events.push_back(c->up_inflight.front().ev);
    c->up_inflight.pop_front();
  }
  while (!c->up_inflight.empty() && hipEventQuery(c->up_inflight.front().ev) == hipSuccess) {
    c->up_events.push_back(c->up_inflight.front().ev);
    c->up_inflight.pop_front();
  }
  std::memcpy(c->up_ring + s, host, bytes);
  SPAMM_HIP(c, hipMemcpyAsync(dev, c->up_ring + s, bytes, hipMemcpyHostToDevice, c->stream));
  hipEvent_t ev = nullptr;
  if (!c->up_events.empty()) {
    ev = c->up_events.back();
    c->up_events.pop_back();
  } else {
    SPAMM_HIP(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  SPAMM_HIP(c, hipEventRecord(ev, c->stream));
  c->up_inflight.push_back({s, e, ev});
  c->up_head = e;
  return SPAMM_OK;
}

spamm_status download(Ctx* c, void* host, const void* dev, size_t bytes) {
  if (bytes == 0) return SPAMM_OK;
  void* st = c->stage(bytes);
  if (!st) return fail(c, SPAMM_EDEVICE, "hipHostMalloc of staging buffer failed");
  SPAMM_HIP(c, hipMemcpyAsync(st, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  SPAMM_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(host, st, bytes);
  return SPAMM_OK;
}

spamm_status nomem(Ctx* c, const char* what, size_t bytes) {
  return fail(c, SPAMM_ENOMEM,
              std::string("arena exhausted allocating ") + what + " (" + std::to_string(bytes) + " bytes, " +
                  std::to_string(c->arena.free_bytes()) + " free)");
}

#define ALLOC(var, bytes, what)                                 \
  do {                                                          \
    (var) = c->alloc(bytes);                                    \
    if (!(var)) return nomem(c, what, size_t(bytes));           \
  } while (0)
// a block that lives only during the call (kept away from the results)
#define ALLOC_TMP(var, bytes, what)                             \
  do {                                                          \
    (var) = c->alloc(bytes, 256, true);                         \
    if (!(var)) return nomem(c, what, size_t(bytes));           \
  } while (0)
// leaf copies are aligned to their leaf size so that a leaf is one index
// from the arena base
#define ALLOC_LEAVES(var, nleaf, leaf_bytes, what)                                      \
  do {                                                                                  \
    (var) = c->alloc(size_t(std::max<int64_t>(nleaf, 1)) * (leaf_bytes), (leaf_bytes)); \
    if (!(var)) return nomem(c, what, size_t(nleaf) * (leaf_bytes));                   \
  } while (0)

// Descriptor tables gathered on the host and sent to the device in one copy
// (one region, one transfer) before the launches that read them.
// A table whose content depends on device addresses inside the set is
// reserved first and written with put() once place() has allocated the set.
struct TableSet {
  std::vector<char> host;
  RegionP dev;
  size_t reserve(size_t bytes) {
    const size_t o = (host.size() + 255) / 256 * 256;
    host.resize(o + bytes);
    return o;
  }
  template <typename T>
  size_t add(const std::vector<T>& v) {
    const size_t o = reserve(v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(host.data() + o, v.data(), v.size() * sizeof(T));
    return o;
  }
  template <typename T>
  void put(size_t off, const std::vector<T>& v) {
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
  }
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(static_cast<char*>(dev->ptr()) + off);
  }
};

spamm_status place_tables(Ctx* c, TableSet& t) {
  if (!t.dev) ALLOC(t.dev, std::max<size_t>(t.host.size(), 256), "descriptor tables");
  return SPAMM_OK;
}

spamm_status send_tables(Ctx* c, TableSet& t) {
  spamm_status st = place_tables(c, t);
  if (st != SPAMM_OK) return st;
  return upload(c, t.dev->ptr(), t.host.data(), t.host.size());
}

// Handle skeleton with the per-level arrays (no leaf storage).
spamm_status new_matrix(Ctx* c, int64_t n, int bs, std::unique_ptr<spamm_mat>& out) {
  auto m = std::make_unique<spamm_mat>();
  m->ctx = c;
  m->n = n;
  m->bs = bs;
  grid_of(n, bs, m->G, m->L);
  if (m->L > kMaxL) return fail(c, SPAMM_EUNSUPPORTED, "quadtree deeper than 11 levels (n/leaf > 2048)");
  const int64_t G2 = int64_t(m->G) * m->G;
  ALLOC(m->slot, G2 * 4, "slot map");
  ALLOC(m->norms, pyramid_size(m->L) * 8, "norm pyramid");
  out = std::move(m);
  return SPAMM_OK;
}

// Row/column views for pruning, computed on first use as an operand (all
// matrices that lack them in one batched pass).  prep_plan allocates the
// views and fills the job table; prep_launch runs it from the device copy.
struct PrepPlan {
  std::vector<PrepJob> jobs;
  int64_t total = 0, waves = 0;
};

spamm_status prep_plan(Ctx* c, const std::vector<spamm_mat*>& mats, PrepPlan& pp) {
  std::vector<spamm_mat*> todo;
  for (spamm_mat* m : mats) {
    if (m->rm_sqrt || std::find(todo.begin(), todo.end(), m) != todo.end()) continue;
    const int64_t G2 = int64_t(m->G) * m->G;
    ALLOC(m->rm_sqrt, G2 * 8, "row view");
    ALLOC(m->rm_slot, G2 * 4, "row slots");
    ALLOC(m->cm_sqrt, G2 * 8, "column view");
    ALLOC(m->cm_slot, G2 * 4, "column slots");
    ALLOC(m->ranges, int64_t(4) * m->G * 4, "ranges");
    PrepJob j;
    j.slot = P<int32_t>(m->slot);
    j.leafnorm = P<double>(m->norms) + level_offset(m->L);
    j.rm_sqrt = P<double>(m->rm_sqrt);
    j.rm_slot = P<int32_t>(m->rm_slot);
    j.cm_sqrt = P<double>(m->cm_sqrt);
    j.cm_slot = P<int32_t>(m->cm_slot);
    j.ranges = P<int32_t>(m->ranges);
    j.base = pp.total;
    j.wbase = pp.waves;
    j.G = m->G;
    j.pad_ = 0;
    pp.jobs.push_back(j);
    todo.push_back(m);
    pp.total += G2;
    pp.waves += 2 * int64_t(m->G);
  }
  return SPAMM_OK;
}

spamm_status prep_launch(Ctx* c, const PrepJob* jd, const PrepPlan& pp) {
  if (pp.jobs.empty()) return SPAMM_OK;
  TimedScope ts(c, kTPrune);
  SPAMM_HIP(c, launch_prep_batch(c->stream, jd, int(pp.jobs.size()), pp.total, pp.waves));
  return SPAMM_OK;
}

// Pyramids over a set of matrices whose leaf level is filled: the job
// table (pyramid_jobs) and its launch from a device copy (it may be
// captured).
std::vector<PyrJob> pyramid_jobs(const std::vector<double*>& norms, const std::vector<int>& Ls) {
  std::vector<PyrJob> jobs(norms.size(), PyrJob{});
  int64_t base = 0;
  for (size_t t = 0; t < norms.size(); ++t) {
    jobs[t].norms = norms[t];
    jobs[t].L = Ls[t];
    jobs[t].sub_levels = std::min(Ls[t], 5);
    jobs[t].block_base = base;
    jobs[t].nsub = int32_t(int64_t(1) << (2 * (Ls[t] - jobs[t].sub_levels)));
    jobs[t].pad_ = 0;
    base += jobs[t].nsub;
  }
  return jobs;
}

spamm_status pyramids_launch(Ctx* c, const PyrJob* jd, const std::vector<PyrJob>& jobs) {
  if (jobs.empty()) return SPAMM_OK;
  TimedScope ts(c, kTPyr);
  SPAMM_HIP(c, launch_pyramid(c->stream, jd, int(jobs.size()), jobs));
  return SPAMM_OK;
}

// keys: an already filled key region (at least nleaf entries) to adopt
spamm_status alloc_store(Ctx* c, Store& s, int64_t nleaf, int bs, uint32_t mask, RegionP keys = nullptr) {
  s.nleaf = nleaf;
  s.bs = bs;
  const size_t e2 = size_t(bs) * bs;
  if (keys) s.keys = keys;
  else ALLOC(s.keys, std::max<int64_t>(nleaf, 1) * 4, "leaf keys");
  if (mask & SPAMM_STORE_F64) ALLOC_LEAVES(s.f64, nleaf, e2 * 8, "FP64 leaves");
  if (mask & SPAMM_STORE_F32) ALLOC_LEAVES(s.f32, nleaf, e2 * 4, "FP32 leaves");
  if (mask & SPAMM_STORE_BF16) {
    ALLOC_LEAVES(s.bf16, nleaf, e2 * 4, "BF16 hi/lo leaves");
    ALLOC_LEAVES(s.bf16t, nleaf, e2 * 4, "transposed BF16 hi/lo leaves");
  }
  return SPAMM_OK;
}

// Make sure the store holds the copies `need` (derived from FP64 if present,
// else from FP32).
spamm_status ensure_store(Ctx* c, Store& s, uint32_t need) {
  const uint32_t missing = need & ~s.mask();
  if (!missing) return SPAMM_OK;
  const size_t e2 = size_t(s.bs) * s.bs;
  RegionP o64, o32, o16, o16t;
  if (missing & SPAMM_STORE_F64) ALLOC_LEAVES(o64, s.nleaf, e2 * 8, "FP64 leaves");
  if (missing & SPAMM_STORE_F32) ALLOC_LEAVES(o32, s.nleaf, e2 * 4, "FP32 leaves");
  if (missing & SPAMM_STORE_BF16) {
    ALLOC_LEAVES(o16, s.nleaf, e2 * 4, "BF16 hi/lo leaves");
    ALLOC_LEAVES(o16t, s.nleaf, e2 * 4, "transposed BF16 hi/lo leaves");
  }
  if (!s.f64 && !s.f32) return fail(c, SPAMM_EUNSUPPORTED, "no FP64/FP32 copy to derive from");
  TimedScope ts(c, kTBuild);
  SPAMM_HIP(c, launch_derive_store(c->stream, s.nleaf, s.bs, P<double>(s.f64), s.f64 ? nullptr : P<float>(s.f32),
                                   P<double>(o64), P<float>(o32), P<uint16_t>(o16), P<uint16_t>(o16t)));
  if (o64) s.f64 = o64;
  if (o32) s.f32 = o32;
  if (o16) {
    s.bf16 = o16;
    s.bf16t = o16t;
  }
  return SPAMM_OK;
}

uint32_t store_for_prec(int prec) {
  switch (prec) {
    case SPAMM_F64: return SPAMM_STORE_F64;
    case SPAMM_F32: return SPAMM_STORE_F32;
    default: return SPAMM_STORE_BF16;
  }
}

bool tau_ok(double t) { return std::isfinite(t) && t >= 0.0; }

// A build's pyramid job table is sent while its first kernels run (before
// the build's read-back), so the copy costs no idle device time.
struct BuildPyr {
  TableSet t;
  size_t off = 0;
  std::vector<PyrJob> jobs;
};

spamm_status send_build_pyr(Ctx* c, const spamm_mat& m, BuildPyr& bp) {
  bp.jobs = pyramid_jobs({P<double>(m.norms)}, {m.L});
  bp.off = bp.t.add(bp.jobs);
  return send_tables(c, bp.t);
}

spamm_status finish_build(Ctx* c, std::unique_ptr<spamm_mat>& m, spamm_mat** out, const BuildPyr& bp) {
  spamm_status st = pyramids_launch(c, bp.t.at<PyrJob>(bp.off), bp.jobs);
  if (st != SPAMM_OK) return st;
  c->live_handles++;
  *out = m.release();
  return SPAMM_OK;
}

// Truncate several (matrix, tau) pairs with one set of launches.  Outputs
// share leaf storage with their inputs; `result` holds 2 doubles per job
// (dropped squared norm, dropped count) on the device.  trunc_plan creates
// the outputs and the job tables (truncation, then the outputs' pyramids);
// trunc_launch runs both from their device copies.
struct TruncPlan {
  std::vector<TruncJob> jobs;
  std::vector<PyrJob> pyr;
  int64_t total = 0;
  RegionP scratch;
  size_t sb = 0;
};

struct TruncIn {
  const spamm_mat* m;
  double tau;
  bool pairs;  // mirror-pair truncation (the symmetric square)
};

spamm_status trunc_plan(Ctx* c, const std::vector<TruncIn>& in, std::vector<std::unique_ptr<spamm_mat>>& out,
                        RegionP& result, TruncPlan& tp) {
  out.clear();
  if (in.empty()) return SPAMM_OK;
  ALLOC(result, in.size() * 16, "truncation results");
  for (size_t t = 0; t < in.size(); ++t) {
    const spamm_mat* a = in[t].m;
    std::unique_ptr<spamm_mat> m;
    spamm_status st = new_matrix(c, a->n, a->bs, m);
    if (st != SPAMM_OK) return st;
    m->store = a->store;
    TruncJob j;
    j.slot = P<int32_t>(a->slot);
    j.leafnorm = P<double>(a->norms) + level_offset(a->L);
    j.out_slot = P<int32_t>(m->slot);
    j.out_norm = P<double>(m->norms) + level_offset(m->L);
    j.result = P<double>(result) + 2 * t;
    j.tau2 = in[t].tau * in[t].tau;
    j.pairs = in[t].pairs ? 1 : 0;
    j.base = tp.total;
    j.G = a->G;
    int kb = 1;
    while ((int64_t(1) << kb) < int64_t(a->G) * a->G) ++kb;
    j.key_bits_lo = kb;
    tp.jobs.push_back(j);
    tp.total += int64_t(a->G) * a->G;
    out.push_back(std::move(m));
  }
  tp.sb = trunc_batch_scratch_bytes(int(tp.jobs.size()), tp.total);
  ALLOC(tp.scratch, tp.sb, "truncation scratch");
  std::vector<double*> nv;
  std::vector<int> lv;
  for (auto& m : out) {
    nv.push_back(P<double>(m->norms));
    lv.push_back(m->L);
  }
  tp.pyr = pyramid_jobs(nv, lv);
  return SPAMM_OK;
}

spamm_status trunc_launch(Ctx* c, const TruncPlan& tp, const TruncJob* jd, const PyrJob* pd) {
  if (tp.jobs.empty()) return SPAMM_OK;
  {
    TimedScope ts(c, kTTrunc);
    SPAMM_HIP(c, launch_trunc_batch(c->stream, jd, int(tp.jobs.size()), tp.total, tp.scratch->ptr(), tp.sb));
  }
  return pyramids_launch(c, pd, tp.pyr);
}

}  // namespace

// ====================================================================== ABI

extern "C" {

const char* spamm_status_string(spamm_status s) {
  switch (s) {
    case SPAMM_OK: return "SPAMM_OK";
    case SPAMM_EINVAL: return "SPAMM_EINVAL";
    case SPAMM_ESHAPE: return "SPAMM_ESHAPE";
    case SPAMM_ENOMEM: return "SPAMM_ENOMEM";
    case SPAMM_ENONFINITE: return "SPAMM_ENONFINITE";
    case SPAMM_EUNSUPPORTED: return "SPAMM_EUNSUPPORTED";
    case SPAMM_EDEVICE: return "SPAMM_EDEVICE";
  }
  return "SPAMM_UNKNOWN";
}

const char* spamm_last_error(const spamm_ctx* ctx) { return ctx ? ctx->c.last_error.c_str() : "no context"; }

spamm_status spamm_ctx_create(int device, void* arena, size_t arena_bytes, spamm_stream stream, spamm_ctx** out) {
  if (!out || !arena || arena_bytes < (size_t(1) << 20) || (reinterpret_cast<uintptr_t>(arena) & 255))
    return SPAMM_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return SPAMM_EDEVICE;
  // the static scratch of spamm_gershgorin_static, once per device
  if (noalloc_setup(device) != hipSuccess) return SPAMM_EDEVICE;
  auto* x = new spamm_ctx;
  x->c.device = device;
  x->c.stream = static_cast<hipStream_t>(stream);
  x->c.arena.init(static_cast<char*>(arena), arena_bytes);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    x->c.n_cu = cus;
  if (const char* e = std::getenv("SPAMM_GEMM_SCHED")) x->c.gemm_sched = std::string(e) == "rm" ? 1 : 0;
  if (!x->c.stage(size_t(1) << 20)) {
    delete x;
    return SPAMM_EDEVICE;
  }
  *out = x;
  return SPAMM_OK;
}

spamm_status spamm_ctx_destroy(spamm_ctx* ctx) {
  if (!ctx) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (c->live_handles != 0) return fail(c, SPAMM_EINVAL, "handles still alive");
  (void)hipStreamSynchronize(c->stream);
  (void)c->collect_timing();
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  for (auto& r : c->up_inflight) (void)hipEventDestroy(r.ev);
  for (hipEvent_t e : c->up_events) (void)hipEventDestroy(e);
  if (c->up_ring) (void)hipHostFree(c->up_ring);
  if (c->host_stage) (void)hipHostFree(c->host_stage);
  if (c->res_host) (void)hipHostFree(c->res_host);
  delete ctx;
  return SPAMM_OK;
}

spamm_status spamm_ctx_set_option(spamm_ctx* ctx, spamm_option key, int64_t value) {
  if (!ctx) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (key == SPAMM_OPT_UNIT_ORDER) {
    if (value < -1 || value > 1024) return fail(c, SPAMM_EINVAL, "unit order: -1 (automatic) or chunk size 0..1024");
    c->gemm_interleave = int(value);
    return SPAMM_OK;
  }
  if (key == SPAMM_OPT_GEMM_QUAD && value == -1) {
    c->gemm_quad = -1;
    return SPAMM_OK;
  }
  if (value != 0 && value != 1) return fail(c, SPAMM_EINVAL, "option value must be 0 or 1");
  switch (key) {
    case SPAMM_OPT_GEMM_TILE: c->gemm_tile = int(value); return SPAMM_OK;
    case SPAMM_OPT_PLACEMENT: c->gemm_sched = int(value); return SPAMM_OK;
    case SPAMM_OPT_GRAPH: c->use_graph = int(value); return SPAMM_OK;
    case SPAMM_OPT_VALIDATE: c->validate = int(value); return SPAMM_OK;
    case SPAMM_OPT_GEMM_QUAD: c->gemm_quad = int(value); return SPAMM_OK;
    default: return fail(c, SPAMM_EINVAL, "unknown option");
  }
}

spamm_status spamm_ctx_get_option(const spamm_ctx* ctx, spamm_option key, int64_t* value) {
  if (!ctx || !value) return SPAMM_EINVAL;
  const Ctx* c = &ctx->c;
  switch (key) {
    case SPAMM_OPT_GEMM_TILE: *value = c->gemm_tile; return SPAMM_OK;
    case SPAMM_OPT_PLACEMENT: *value = c->gemm_sched; return SPAMM_OK;
    case SPAMM_OPT_GRAPH: *value = c->use_graph; return SPAMM_OK;
    case SPAMM_OPT_UNIT_ORDER: *value = c->gemm_interleave; return SPAMM_OK;
    case SPAMM_OPT_VALIDATE: *value = c->validate; return SPAMM_OK;
    case SPAMM_OPT_GEMM_QUAD: *value = c->gemm_quad; return SPAMM_OK;
    default: return SPAMM_EINVAL;
  }
}

spamm_status spamm_ctx_set_stream(spamm_ctx* ctx, spamm_stream stream) {
  if (!ctx) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  SPAMM_HIP(c, hipStreamSynchronize(c->stream));
  c->stream = static_cast<hipStream_t>(stream);
  return SPAMM_OK;
}

spamm_status spamm_ctx_timing(spamm_ctx* ctx, int32_t enable, int32_t reset, spamm_timing* out) {
  if (!ctx) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (out) {
    SPAMM_HIP(c, c->collect_timing());
    out->build_ms = c->t_ms[kTBuild];
    out->trunc_ms = c->t_ms[kTTrunc];
    out->prune_ms = c->t_ms[kTPrune];
    out->gemm_ms = c->t_ms[kTGemm];
    out->pyramid_ms = c->t_ms[kTPyr];
    out->build_launches = c->t_cnt[kTBuild];
    out->trunc_launches = c->t_cnt[kTTrunc];
    out->prune_launches = c->t_cnt[kTPrune];
    out->gemm_launches = c->t_cnt[kTGemm];
    out->pyramid_launches = c->t_cnt[kTPyr];
    out->gemm_flops = c->gemm_flops;
    out->gemm_quad_launches = c->gemm_quad_launches;
  }
  if (reset) {
    SPAMM_HIP(c, c->collect_timing());
    for (int k = 0; k < kTClasses; ++k) {
      c->t_ms[k] = 0.0;
      c->t_cnt[k] = 0;
    }
    c->gemm_flops = 0.0;
    c->gemm_quad_launches = 0;
  }
  c->timing = enable != 0;
  return SPAMM_OK;
}

spamm_status spamm_ctx_arena_info(const spamm_ctx* ctx, size_t* used, size_t* free_bytes, size_t* largest_free) {
  if (!ctx) return SPAMM_EINVAL;
  if (used) *used = ctx->c.arena.used();
  if (free_bytes) *free_bytes = ctx->c.arena.free_bytes();
  if (largest_free) *largest_free = ctx->c.arena.largest_free();
  return SPAMM_OK;
}

spamm_status spamm_build(spamm_ctx* ctx, const double* dense, int64_t n, int64_t ld, int32_t leaf, uint32_t stores,
                         spamm_mat** out) {
  if (!ctx || !out) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  *out = nullptr;
  if (!dense || n < 1 || ld < n || !leaf_ok(leaf)) return fail(c, SPAMM_EINVAL, "bad build arguments");
  if (stores == 0 || (stores & ~7u)) return fail(c, SPAMM_EINVAL, "bad store mask");
  std::unique_ptr<spamm_mat> m;
  spamm_status st = new_matrix(c, n, leaf, m);
  if (st != SPAMM_OK) return st;
  const int64_t G2 = int64_t(m->G) * m->G;
  RegionP flag, total, scratch, nf, keys;
  ALLOC(flag, G2 * 4, "flags");
  ALLOC(nf, 256, "flags");
  ALLOC(keys, G2 * 4, "leaf keys");
  const size_t sb = scan_scratch_bytes(G2);
  ALLOC(scratch, sb, "scan scratch");
  int64_t* tot = reinterpret_cast<int64_t*>(static_cast<char*>(nf->ptr()) + 64);
  {
  TimedScope ts(c, kTBuild);
  SPAMM_HIP(c, launch_zero_i32(c->stream, P<int32_t>(nf), 4));
  SPAMM_HIP(c, launch_build_scan_dense(c->stream, dense, n, ld, leaf, m->G, P<double>(m->norms) + level_offset(m->L),
                                       P<int32_t>(flag), P<int32_t>(nf)));
  SPAMM_HIP(c, launch_flags_to_slots(c->stream, P<int32_t>(flag), G2, P<int32_t>(m->slot), P<int32_t>(keys), tot,
                                     scratch->ptr(), sb));
  }
  BuildPyr bp;
  st = send_build_pyr(c, *m, bp);
  if (st != SPAMM_OK) return st;
  struct {
    int32_t nf;
    int32_t pad[15];
    int64_t total;
  } hb;
  st = download(c, &hb, nf->ptr(), sizeof(hb));
  if (st != SPAMM_OK) return st;
  if (hb.nf) return fail(c, SPAMM_ENONFINITE, "NaN or Inf in the input matrix");
  m->nonnull = hb.total;
  m->store = std::make_shared<Store>();
  st = alloc_store(c, *m->store, hb.total, leaf, stores, keys);
  if (st != SPAMM_OK) return st;
  TimedScope ts2(c, kTBuild);
  SPAMM_HIP(c, launch_copy_dense_leaves(c->stream, dense, n, ld, leaf, hb.total, P<int32_t>(m->store->keys),
                                        P<double>(m->store->f64), P<float>(m->store->f32),
                                        P<uint16_t>(m->store->bf16), P<uint16_t>(m->store->bf16t)));
  return finish_build(c, m, out, bp);
}

spamm_status spamm_build_blocks_batch(spamm_ctx* ctx, int32_t count, const spamm_block_list* lists,
                                      spamm_mat** out) {
  if (!ctx) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (count < 0 || (count > 0 && (!lists || !out))) return fail(c, SPAMM_EINVAL, "bad build_blocks arguments");
  for (int t = 0; t < count; ++t) out[t] = nullptr;
  for (int t = 0; t < count; ++t) {
    const spamm_block_list& b = lists[t];
    if (b.n < 1 || !leaf_ok(b.leaf) || b.nblocks < 0 || (b.nblocks > 0 && (!b.coords || !b.data)))
      return fail(c, SPAMM_EINVAL, "bad build_blocks arguments");
    if (b.stores == 0 || (b.stores & ~7u)) return fail(c, SPAMM_EINVAL, "bad store mask");
    if (b.nblocks > INT32_MAX) return fail(c, SPAMM_EINVAL, "too many blocks");
  }
  if (count == 0) return SPAMM_OK;
  // Every list's leaf store has one slot per listed block (block t is leaf
  // slot t), so one pass over the blocks computes the norms and null flags
  // and writes the slot map, the keys and the leaf copies: one set of
  // launches for all lists, one read-back of every list's error bits and
  // leaf count, and the pyramids queued after it.
  struct Hdr {
    int32_t err;
    int32_t pad[15];
    int64_t total;
    int64_t pad2[7];
  };
  static_assert(sizeof(Hdr) == 128, "one header per list");
  std::vector<std::unique_ptr<spamm_mat>> ms(count);
  std::vector<RegionP> src(count);
  std::vector<BuildJob> jobs(count);
  RegionP hdr;
  ALLOC(hdr, int64_t(count) * sizeof(Hdr), "build headers");
  int64_t g2_total = 0, blocks_total = 0;
  for (int t = 0; t < count; ++t) {
    const spamm_block_list& b = lists[t];
    spamm_status st = new_matrix(c, b.n, b.leaf, ms[t]);
    if (st != SPAMM_OK) return st;
    spamm_mat* m = ms[t].get();
    const int64_t G2 = int64_t(m->G) * m->G;
    ALLOC(src[t], G2 * 4, "block index");
    m->store = std::make_shared<Store>();
    st = alloc_store(c, *m->store, std::max<int64_t>(b.nblocks, 1), b.leaf, b.stores);
    if (st != SPAMM_OK) return st;
    BuildJob& J = jobs[t];
    std::memset(&J, 0, sizeof(J));
    J.n = b.n;
    J.bs = b.leaf;
    J.G = m->G;
    J.nblocks = b.nblocks;
    J.coords = b.coords;
    J.data = b.data;
    J.src_of = P<int32_t>(src[t]);
    J.leafnorm = P<double>(m->norms) + level_offset(m->L);
    J.slot = P<int32_t>(m->slot);
    J.keys = P<int32_t>(m->store->keys);
    J.err = &(P<Hdr>(hdr) + t)->err;
    J.total = &(P<Hdr>(hdr) + t)->total;
    J.f64 = P<double>(m->store->f64);
    J.f32 = P<float>(m->store->f32);
    J.b16 = P<uint16_t>(m->store->bf16);
    J.b16t = P<uint16_t>(m->store->bf16t);
    J.g2_base = g2_total;
    J.blk_base = blocks_total;
    g2_total += G2;
    blocks_total += b.nblocks;
  }
  if (blocks_total > INT32_MAX || g2_total > INT32_MAX)
    return fail(c, SPAMM_EINVAL, "too many blocks in one build call");
  std::vector<PyrJob> pjobs;
  {
    std::vector<double*> nv;
    std::vector<int> lv;
    for (auto& m : ms) {
      nv.push_back(P<double>(m->norms));
      lv.push_back(m->L);
    }
    pjobs = pyramid_jobs(nv, lv);
  }
  TableSet tabs;
  const size_t oj = tabs.add(jobs), po = tabs.add(pjobs);
  spamm_status st = send_tables(c, tabs);
  if (st != SPAMM_OK) return st;
  {
    TimedScope ts(c, kTBuild);
    SPAMM_HIP(c, launch_build_batch(c->stream, tabs.at<BuildJob>(oj), count, g2_total, blocks_total));
  }
  std::vector<Hdr> hb(count);
  st = download(c, hb.data(), hdr->ptr(), int64_t(count) * sizeof(Hdr));
  if (st != SPAMM_OK) return st;
  for (int t = 0; t < count; ++t) {
    const int32_t e = hb[t].err;
    if (e & 1) return fail(c, SPAMM_EINVAL, "block coordinate outside the matrix");
    if (e & 2) return fail(c, SPAMM_EINVAL, "block coordinate listed twice");
    if (e & 4) return fail(c, SPAMM_EINVAL, "non-zero entry past row/column n");
    if (e & 8) return fail(c, SPAMM_ENONFINITE, "NaN or Inf in the input blocks");
  }
  st = pyramids_launch(c, tabs.at<PyrJob>(po), pjobs);
  if (st != SPAMM_OK) return st;
  for (int t = 0; t < count; ++t) {
    ms[t]->nonnull = hb[t].total;
    c->live_handles++;
    out[t] = ms[t].release();
  }
  return SPAMM_OK;
}

spamm_status spamm_build_blocks(spamm_ctx* ctx, int64_t n, int32_t leaf, int64_t nblocks, const int32_t* coords,
                                const double* data, uint32_t stores, spamm_mat** out) {
  if (!ctx || !out) return SPAMM_EINVAL;
  *out = nullptr;
  const spamm_block_list b{n, leaf, stores, nblocks, coords, data};
  return spamm_build_blocks_batch(ctx, 1, &b, out);
}

static spamm_status truncate_one(spamm_ctx* ctx, const spamm_mat* in, double tau, bool pairs, spamm_mat** out,
                                 double* dropped_sq) {
  if (!ctx || !out) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  *out = nullptr;
  if (!in || in->ctx != c) return fail(c, SPAMM_EINVAL, "bad matrix handle");
  if (!tau_ok(tau)) return fail(c, SPAMM_EINVAL, "tau must be finite and >= 0");
  std::vector<std::unique_ptr<spamm_mat>> ms;
  RegionP res;
  TruncPlan tp;
  spamm_status st = trunc_plan(c, {{in, tau, pairs}}, ms, res, tp);
  if (st != SPAMM_OK) return st;
  TableSet tabs;
  const size_t oj = tabs.add(tp.jobs), op = tabs.add(tp.pyr);
  st = send_tables(c, tabs);
  if (st != SPAMM_OK) return st;
  st = trunc_launch(c, tp, tabs.at<TruncJob>(oj), tabs.at<PyrJob>(op));
  if (st != SPAMM_OK) return st;
  double hr[2];
  st = download(c, hr, res->ptr(), sizeof(hr));
  if (st != SPAMM_OK) return st;
  if (dropped_sq) *dropped_sq = hr[0];
  ms[0]->nonnull = (in->nonnull >= 0) ? in->nonnull - int64_t(hr[1]) : -1;
  c->live_handles++;
  *out = ms[0].release();
  return SPAMM_OK;
}

spamm_status spamm_truncate(spamm_ctx* ctx, const spamm_mat* in, double tau, spamm_mat** out, double* dropped_sq) {
  return truncate_one(ctx, in, tau, false, out, dropped_sq);
}

spamm_status spamm_truncate_symmetric(spamm_ctx* ctx, const spamm_mat* in, double tau, spamm_mat** out,
                                      double* dropped_sq) {
  return truncate_one(ctx, in, tau, true, out, dropped_sq);
}

spamm_status spamm_truncate_elementwise(spamm_ctx* ctx, const spamm_mat* in, double tau, spamm_mat** out,
                                        double* dropped_sq) {
  if (!ctx || !out) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  *out = nullptr;
  if (!in || in->ctx != c) return fail(c, SPAMM_EINVAL, "bad matrix handle");
  if (!tau_ok(tau)) return fail(c, SPAMM_EINVAL, "tau must be finite and >= 0");
  if (!in->store || !in->store->f64)
    return fail(c, SPAMM_EUNSUPPORTED, "element-wise truncation needs the FP64 copy of the matrix");
  std::unique_ptr<spamm_mat> m;
  spamm_status st = new_matrix(c, in->n, in->bs, m);
  if (st != SPAMM_OK) return st;
  m->store = std::make_shared<Store>();
  // same slots as the input, so the keys are shared (they never change)
  st = alloc_store(c, *m->store, in->store->nleaf, in->bs, in->store->mask(), in->store->keys);
  if (st != SPAMM_OK) return st;
  const int64_t G2 = int64_t(m->G) * m->G;
  RegionP dropped, part, hdr;
  ALLOC(dropped, G2 * 8, "dropped norms");
  ALLOC(part, ((G2 + 4095) / 4096) * 8, "partial sums");
  ALLOC(hdr, 16, "count and total");
  ElemTruncJob j;
  j.G = m->G;
  j.bs = m->bs;
  j.tau = tau;
  j.in_slot = P<int32_t>(in->slot);
  j.in_f64 = P<double>(in->store->f64);
  j.slot = P<int32_t>(m->slot);
  j.leafnorm = P<double>(m->norms) + level_offset(m->L);
  j.dropped = P<double>(dropped);
  j.count = P<int64_t>(hdr);
  j.f64 = P<double>(m->store->f64);
  j.f32 = P<float>(m->store->f32);
  j.b16 = P<uint16_t>(m->store->bf16);
  j.b16t = P<uint16_t>(m->store->bf16t);
  SPAMM_HIP(c, launch_zero_i32(c->stream, P<int32_t>(hdr), 2));
  {
    TimedScope ts(c, kTTrunc);
    SPAMM_HIP(c, launch_trunc_elem(c->stream, j));
    SPAMM_HIP(c, launch_sum_f64(c->stream, P<double>(dropped), G2, P<double>(part), P<double>(hdr) + 1));
  }
  const std::vector<PyrJob> pj = pyramid_jobs({P<double>(m->norms)}, {m->L});
  TableSet tabs;
  const size_t po = tabs.add(pj);
  st = send_tables(c, tabs);
  if (st != SPAMM_OK) return st;
  st = pyramids_launch(c, tabs.at<PyrJob>(po), pj);
  if (st != SPAMM_OK) return st;
  struct {
    int64_t count;
    double dropped;
  } h;
  st = download(c, &h, hdr->ptr(), sizeof(h));
  if (st != SPAMM_OK) return st;
  if (dropped_sq) *dropped_sq = h.dropped;
  m->nonnull = h.count;
  c->live_handles++;
  *out = m.release();
  return SPAMM_OK;
}

static spamm_status multiply_core(Ctx* c, int32_t count, const spamm_request* reqs, spamm_mat** C_out,
                                  spamm_stats* st_out);

// With validation on, every product that is not FP64 gets an FP64 twin (same
// operands, tau, mode and epilogue) in the same batch.  The twin shares the
// truncations and the norm tests, so it keeps the same products and its C
// holds the same non-null leaves in the same slots; the two C stores are
// then compared leaf slot by leaf slot and the twin is released.
spamm_status spamm_multiply_batch(spamm_ctx* ctx, int32_t count, const spamm_request* reqs, spamm_mat** C_out,
                                  spamm_stats* st_out) {
  if (!ctx) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (!c->validate || count <= 0 || !reqs || !C_out) {
    const spamm_status st = multiply_core(c, count, reqs, C_out, st_out);
    if (st == SPAMM_OK && st_out)
      for (int r = 0; r < count; ++r) st_out[r].val_err = -1.0;
    return st;
  }
  for (int r = 0; r < count; ++r) C_out[r] = nullptr;
  std::vector<spamm_request> all(reqs, reqs + count);
  std::vector<int> twin(count, -1);
  for (int r = 0; r < count; ++r) {
    const spamm_request& q = reqs[r];
    if (q.prec == SPAMM_F64 || !q.A || !q.B || q.A->ctx != c || q.B->ctx != c) continue;  // core checks handles
    if (!q.A->store || !q.A->store->f64 || !q.B->store || !q.B->store->f64)
      return fail(c, SPAMM_EUNSUPPORTED, "validation needs the FP64 copy of A and B");
    twin[r] = int(all.size());
    spamm_request t = q;
    t.prec = SPAMM_F64;
    all.push_back(t);
  }
  const int total = int(all.size());
  std::vector<spamm_mat*> Cs(total, nullptr);
  std::vector<spamm_stats> sts(total);
  spamm_status st = multiply_core(c, total, all.data(), Cs.data(), st_out ? sts.data() : nullptr);
  if (st != SPAMM_OK) return st;
  auto release_all = [&]() {
    for (spamm_mat* m : Cs) (void)spamm_release(ctx, m);
  };
  std::vector<ValJob> jobs;
  std::vector<int> job_of(count, -1);
  int64_t nchunks = 0;
  for (int r = 0; r < count; ++r) {
    if (twin[r] < 0) continue;
    const spamm_mat* C = Cs[r];
    const spamm_mat* T = Cs[twin[r]];
    if (C->nonnull != T->nonnull) {
      release_all();
      return fail(c, SPAMM_EDEVICE, "validation twin kept different products");
    }
    ValJob j;
    j.c32 = C->nonnull ? P<float>(C->store->f32) : nullptr;
    j.c64 = T->nonnull ? P<double>(T->store->f64) : nullptr;
    j.nelem = C->nonnull * int64_t(C->bs) * C->bs;
    j.chunk_base = nchunks;
    nchunks += (j.nelem + kValChunk - 1) / kValChunk;
    job_of[r] = int(jobs.size());
    jobs.push_back(j);
  }
  if (!jobs.empty()) {
    TableSet tabs;
    const size_t oj = tabs.add(jobs);
    RegionP part = c->alloc(size_t(std::max<int64_t>(nchunks, 1)) * 8);
    if (!part) {
      release_all();
      return nomem(c, "validation partial sums", size_t(std::max<int64_t>(nchunks, 1)) * 8);
    }
    st = send_tables(c, tabs);
    if (st == SPAMM_OK && !c->results(jobs.size() * sizeof(double)))
      st = fail(c, SPAMM_EDEVICE, "mapped results buffer");
    if (st == SPAMM_OK) {
      const hipError_t e = launch_validate(c->stream, tabs.at<ValJob>(oj), int(jobs.size()), nchunks,
                                           P<double>(part), reinterpret_cast<double*>(c->res_dev));
      if (e != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
        st = fail(c, SPAMM_EDEVICE, std::string("validation: ") + hipGetErrorString(hipGetLastError()));
    }
    if (st != SPAMM_OK) {
      release_all();
      return st;
    }
  }
  const double* vsq = reinterpret_cast<const double*>(c->res_host);
  for (int r = 0; r < count; ++r) {
    C_out[r] = Cs[r];
    Cs[r] = nullptr;
    if (st_out) {
      st_out[r] = sts[r];
      st_out[r].val_err = twin[r] < 0 ? 0.0 : std::sqrt(vsq[job_of[r]]);
    }
  }
  release_all();  // the twins
  return SPAMM_OK;
}

static spamm_status multiply_core(Ctx* c, int32_t count, const spamm_request* reqs, spamm_mat** C_out,
                                  spamm_stats* st_out) {
  if (count < 0 || (count > 0 && (!reqs || !C_out))) return fail(c, SPAMM_EINVAL, "bad batch arguments");
  for (int r = 0; r < count; ++r) C_out[r] = nullptr;
  if (count == 0) return SPAMM_OK;

  // ---- validate
  for (int r = 0; r < count; ++r) {
    const spamm_request& q = reqs[r];
    if (!q.A || !q.B || q.A->ctx != c || q.B->ctx != c) return fail(c, SPAMM_EINVAL, "bad matrix handle");
    if (q.A->n != q.B->n || q.A->bs != q.B->bs) return fail(c, SPAMM_ESHAPE, "A and B differ in n or leaf size");
    if (!tau_ok(q.tau)) return fail(c, SPAMM_EINVAL, "tau must be finite and >= 0");
    if (q.mode < 0 || q.mode > 4) return fail(c, SPAMM_EINVAL, "bad mode");
    if ((q.mode == SPAMM_SPAMM_SYM || q.mode == SPAMM_HYBRID_SYM) && q.A != q.B)
      return fail(c, SPAMM_EINVAL, "the symmetric square needs B = A (the same handle)");
    if (q.prec < 0 || q.prec > 3) return fail(c, SPAMM_EINVAL, "bad precision");
    if (!gemm_supported(q.prec, q.A->bs)) return fail(c, SPAMM_EUNSUPPORTED, "precision/leaf size not built");
    if (q.A->G > (1 << (kUnitTileShift / 2)))
      return fail(c, SPAMM_EUNSUPPORTED, "more than 16384 leaf rows");
    if (q.ep) {
      if (q.ep->D && (q.ep->D->ctx != c)) return fail(c, SPAMM_EINVAL, "bad epilogue matrix");
      if (q.ep->D && (q.ep->D->n != q.A->n || q.ep->D->bs != q.A->bs))
        return fail(c, SPAMM_ESHAPE, "D differs in n or leaf size");
      if (!std::isfinite(q.ep->alpha) || !std::isfinite(q.ep->beta))
        return fail(c, SPAMM_EINVAL, "alpha/beta must be finite");
    }
  }

  // ---- truncations (one per distinct (matrix, tau) in the batch, all at once)
  // one truncation per distinct (matrix, tau, pair form)
  std::map<std::tuple<const spamm_mat*, uint64_t, bool>, int> tindex;
  std::vector<TruncIn> tjobs;
  auto tkey = [](const spamm_mat* m, double tau, bool pairs) {
    uint64_t bits;
    std::memcpy(&bits, &tau, 8);
    return std::make_tuple(m, bits, pairs);
  };
  for (int r = 0; r < count; ++r) {
    const spamm_request& q = reqs[r];
    if (q.mode == SPAMM_SPAMM || q.mode == SPAMM_SPAMM_SYM) continue;  // no truncation
    const bool pairs = q.mode == SPAMM_HYBRID_SYM;
    for (const spamm_mat* m : {q.A, q.B}) {
      auto k = tkey(m, q.tau, pairs);
      if (!tindex.count(k)) {
        tindex[k] = int(tjobs.size());
        tjobs.push_back({m, q.tau, pairs});
      }
    }
  }
  // every table the launches up to the counting pass read is planned on the
  // host first and sent in one copy
  std::vector<std::unique_ptr<spamm_mat>> tmats;
  RegionP tres;
  TruncPlan tplan;
  {
    spamm_status st = trunc_plan(c, tjobs, tmats, tres, tplan);
    if (st != SPAMM_OK) return st;
  }
  std::vector<spamm_mat*> Au(count), Bu(count);
  std::vector<const double*> trA(count, nullptr), trB(count, nullptr);
  std::vector<spamm_mat*> operands;
  for (int r = 0; r < count; ++r) {
    const spamm_request& q = reqs[r];
    if (q.mode == SPAMM_SPAMM || q.mode == SPAMM_SPAMM_SYM) {
      Au[r] = const_cast<spamm_mat*>(q.A);
      Bu[r] = const_cast<spamm_mat*>(q.B);
    } else {
      const bool pairs = q.mode == SPAMM_HYBRID_SYM;
      const int ia = tindex[tkey(q.A, q.tau, pairs)], ib = tindex[tkey(q.B, q.tau, pairs)];
      Au[r] = tmats[ia].get();
      Bu[r] = tmats[ib].get();
      trA[r] = P<double>(tres) + 2 * ia;
      trB[r] = P<double>(tres) + 2 * ib;
    }
    operands.push_back(Au[r]);
    operands.push_back(Bu[r]);
  }
  PrepPlan pplan;
  {
    spamm_status st = prep_plan(c, operands, pplan);
    if (st != SPAMM_OK) return st;
  }
  for (int r = 0; r < count; ++r) {
    const spamm_request& q = reqs[r];
    spamm_status st = ensure_store(c, *Au[r]->store, store_for_prec(q.prec));
    if (st != SPAMM_OK) return st;
    st = ensure_store(c, *Bu[r]->store, store_for_prec(q.prec));
    if (st != SPAMM_OK) return st;
    if (q.ep && q.ep->D) {
      st = ensure_store(c, *q.ep->D->store, q.prec == SPAMM_F64 ? SPAMM_STORE_F64 : SPAMM_STORE_F32);
      if (st != SPAMM_OK) return st;
    }
  }

  // ---- descriptors and counting pass
  std::vector<ReqDev> rd(count);
  int64_t total_c = 0, total_chunks = 0;
  bool any_sym = false;
  for (int r = 0; r < count; ++r) {
    const spamm_request& q = reqs[r];
    ReqDev& d = rd[r];
    std::memset(&d, 0, sizeof(d));
    auto md = [](spamm_mat* m) {
      MatDev x;
      x.slot = P<int32_t>(m->slot);
      x.leafnorm = P<double>(m->norms) + level_offset(m->L);
      x.rm_sqrt = P<double>(m->rm_sqrt);
      x.rm_slot = P<int32_t>(m->rm_slot);
      x.cm_sqrt = P<double>(m->cm_sqrt);
      x.cm_slot = P<int32_t>(m->cm_slot);
      x.ranges = P<int32_t>(m->ranges);
      x.G = m->G;
      x.L = m->L;
      return x;
    };
    d.A = md(Au[r]);
    d.B = md(Bu[r]);
    d.slotD = (q.ep && q.ep->D) ? P<int32_t>(q.ep->D->slot) : nullptr;
    d.tau = q.tau;
    d.use_norms = q.mode != SPAMM_TRUNCMUL;
    d.sym = q.mode == SPAMM_SPAMM_SYM || q.mode == SPAMM_HYBRID_SYM;
    any_sym = any_sym || d.sym;
    d.G = q.A->G;
    d.L = q.A->L;
    d.bs = q.A->bs;
    d.cbase = total_c;
    d.prec = q.prec;
    d.rootA = P<double>(q.A->norms);
    d.rootB = P<double>(q.B->norms);
    d.rootAu = P<double>(Au[r]->norms);
    d.truncA = trA[r];
    d.truncB = trB[r];
    d.stat_base = total_chunks;
    total_c += int64_t(d.G) * d.G;
    total_chunks += (int64_t(d.G) * d.G + kStatChunk - 1) / kStatChunk;
  }
  // packed counts: the kept count of a C leaf is at most G (one per k), so
  // the batch's kept total is below sum G^3 and its non-null total at most
  // total_c; both fields of the scanned int64 must fit
  int cnt_bits = 1, c_bits = 1;
  {
    int64_t ub = 0;
    for (int r = 0; r < count; ++r) ub += int64_t(rd[r].G) * rd[r].G * rd[r].G;
    while ((int64_t(1) << cnt_bits) <= ub) ++cnt_bits;
    while ((int64_t(1) << c_bits) <= total_c) ++c_bits;
    if (cnt_bits + c_bits > 62)
      return fail(c, SPAMM_EUNSUPPORTED, "batch too large for one counting pass; split it");
  }
  // per-request totals and statistics come back through mapped host memory
  const size_t res_tot = (size_t(count) * sizeof(ReqTotals) + 255) / 256 * 256;
  if (!c->results(res_tot + size_t(count) * sizeof(ReqStatsDev)))
    return fail(c, SPAMM_EDEVICE, "hipHostMalloc of the result buffer failed");
  ReqTotals* totals_h = reinterpret_cast<ReqTotals*>(c->res_host);
  ReqTotals* totals_d = reinterpret_cast<ReqTotals*>(c->res_dev);
  RegionP packed, scanned, bnd_all, cand_all, pb_all, scan_scr;
  ALLOC_TMP(packed, total_c * 8, "counts");
  ALLOC_TMP(scanned, (total_c + 1) * 8, "offsets");
  ALLOC_TMP(bnd_all, total_c * 8, "bounds");
  ALLOC_TMP(cand_all, total_c * 4, "candidates");
  ALLOC_TMP(pb_all, total_c * 8, "rounding bounds");
  const size_t ssb = scan_scratch_bytes(total_c);
  ALLOC_TMP(scan_scr, ssb, "scan scratch");
  // symmetric squares: one flag per request, set on the device when the
  // operand's (or D's) null map is not symmetric
  RegionP symflags;
  if (any_sym) {
    ALLOC_TMP(symflags, int64_t(count) * 4, "symmetry flags");
    for (int r = 0; r < count; ++r) rd[r].asym = P<int32_t>(symflags) + r;
  }
  TableSet pre;
  const size_t o_tj = pre.add(tplan.jobs), o_tp = pre.add(tplan.pyr), o_pj = pre.add(pplan.jobs),
               o_rd = pre.add(rd);
  spamm_status st = send_tables(c, pre);
  if (st != SPAMM_OK) return st;
  st = trunc_launch(c, tplan, pre.at<TruncJob>(o_tj), pre.at<PyrJob>(o_tp));
  if (st != SPAMM_OK) return st;
  st = prep_launch(c, pre.at<PrepJob>(o_pj), pplan);
  if (st != SPAMM_OK) return st;
  {
  TimedScope ts(c, kTPrune);
  if (any_sym) {  // after the truncations, before the counting pass reads the flags
    SPAMM_HIP(c, launch_zero_i32(c->stream, P<int32_t>(symflags), count));
    for (int r = 0; r < count; ++r)
      if (rd[r].sym)
        SPAMM_HIP(c, launch_sym_check(c->stream, rd[r].G, rd[r].A.slot, rd[r].slotD, P<int32_t>(symflags) + r));
  }
  const ReqDev* rd0 = pre.at<ReqDev>(o_rd);
  SPAMM_HIP(c, launch_prune_count(c->stream, rd0, count, total_c, cnt_bits, P<int64_t>(packed), P<double>(bnd_all),
                                  P<int32_t>(cand_all), P<double>(pb_all)));
  SPAMM_HIP(c, launch_scan_i64(c->stream, P<int64_t>(packed), P<int64_t>(scanned), total_c, scan_scr->ptr(), ssb));
  SPAMM_HIP(c, launch_gather_totals(c->stream, rd0, count, cnt_bits, P<int64_t>(scanned), totals_d));
  }
  // the parts of every C whose size does not depend on the counts are set up
  // while the counting pass runs
  std::vector<std::unique_ptr<spamm_mat>> Cs(count);
  std::vector<RegionP> cand_r(count), trace_r(count);
  for (int r = 0; r < count; ++r) {
    const spamm_request& q = reqs[r];
    st = new_matrix(c, q.A->n, q.A->bs, Cs[r]);
    if (st != SPAMM_OK) return st;
    spamm_mat* C = Cs[r].get();
    const int64_t G2 = int64_t(C->G) * C->G;
    ALLOC(C->plan_off, (G2 + 1) * 8, "plan offsets");
    ALLOC(C->plan_bnd, G2 * 8, "skipped bounds");
    ALLOC_TMP(cand_r[r], G2 * 4, "candidate counts");
    ALLOC_TMP(trace_r[r], int64_t(C->G) * 8, "trace parts");
    C->store = std::make_shared<Store>();
    C->plan_Astore = Au[r]->store;
    C->plan_Bstore = Bu[r]->store;
  }
  RegionP part;
  if (st_out) ALLOC_TMP(part, total_chunks * sizeof(StatPartial), "stat partials");
  SPAMM_HIP(c, hipStreamSynchronize(c->stream));
  const std::vector<ReqTotals> ht(totals_h, totals_h + count);
  // the partial statistics need only the counting pass: they run while the
  // host lays out the results
  if (st_out) {
    TimedScope ts(c, kTPrune);
    SPAMM_HIP(c, launch_stats_partial(c->stream, pre.at<ReqDev>(o_rd), count, total_chunks, P<double>(bnd_all),
                                      P<int32_t>(cand_all), P<double>(pb_all), P<StatPartial>(part)));
  }

  // ---- allocate results; work units grouped by (precision, leaf size)
  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int r = 0; r < count; ++r) groups[{reqs[r].prec, reqs[r].A->bs}].push_back(r);
  int64_t wu_total = 0;
  std::vector<std::pair<std::pair<int, int>, std::pair<int64_t, int64_t>>> launches;
  for (auto& gk : groups) {
    const int64_t start = wu_total;
    for (int r : gk.second) {
      rd[r].wu_base = wu_total;
      wu_total += ht[r].c_nonnull * gemm_unit_tiles(gk.first.second);
    }
    launches.push_back({gk.first, {start, wu_total - start}});
  }
  for (int r = 0; r < count; ++r) {
    const spamm_request& q = reqs[r];
    ReqDev& d = rd[r];
    spamm_mat* C = Cs[r].get();
    const int64_t nk = ht[r].n_kept, cn = ht[r].c_nonnull;
    C->nonnull = cn;
    C->n_kept = nk;
    st = alloc_store(c, *C->store, cn, C->bs, q.prec == SPAMM_F64 ? SPAMM_STORE_F64 : SPAMM_STORE_F32);
    if (st != SPAMM_OK) return st;
    ALLOC(C->plan_pairs, std::max<int64_t>(nk, 1) * 8, "plan pairs");
    d.pairs = P<int2>(C->plan_pairs);
    d.pk = nullptr;
    d.qbase = 0;
    d.off = P<int64_t>(C->plan_off);
    d.cslot = P<int32_t>(C->slot);
    d.ckeys = P<int32_t>(C->store->keys);
    d.cnorm = P<double>(C->norms);
    d.bnd = P<double>(C->plan_bnd);
    d.ncand = P<int32_t>(cand_r[r]);
    d.trace_part = P<double>(trace_r[r]);
    d.cstore = q.prec == SPAMM_F64 ? C->store->f64->ptr() : C->store->f32->ptr();
    // operands, pairs and C leaves as indices from the arena base
    const char* base = c->arena.base();
    const Store& as = *Au[r]->store;
    const Store& bs = *Bu[r]->store;
    const size_t e2 = size_t(q.A->bs) * q.A->bs;
    const void *Ap, *Bp;
    size_t lb;
    switch (q.prec) {
      case SPAMM_F64:
        Ap = as.f64->ptr();
        Bp = bs.f64->ptr();
        lb = e2 * 8;
        break;
      case SPAMM_F32:
        Ap = as.f32->ptr();
        Bp = bs.f32->ptr();
        lb = e2 * 4;
        break;
      default:
        Ap = as.bf16->ptr();
        Bp = bs.bf16t->ptr();
        lb = e2 * 4;
    }
    const size_t lc = e2 * (q.prec == SPAMM_F64 ? 8 : 4);
    const size_t ao = static_cast<const char*>(Ap) - base, bo = static_cast<const char*>(Bp) - base;
    const size_t co = static_cast<const char*>(d.cstore) - base, po = reinterpret_cast<const char*>(d.pairs) - base;
    if (ao % lb || bo % lb || co % lc || po % 8) return fail(c, SPAMM_EDEVICE, "leaf store not aligned in the arena");
    d.aoff = int64_t(ao / lb);
    d.boff = int64_t(bo / lb);
    d.cidx = int64_t(co / lc);
    d.pairs_idx = int64_t(po / 8);
    if (d.aoff + as.nleaf > INT32_MAX || d.boff + bs.nleaf > INT32_MAX || d.cidx + cn > INT32_MAX)
      return fail(c, SPAMM_EUNSUPPORTED, "arena too large for 32-bit leaf indices at this leaf size");
    C->plan_aoff = d.aoff;
    if (q.ep) {
      d.use_ep = 1;
      d.alpha = q.ep->alpha;
      d.beta = q.ep->beta;
      if (q.ep->D) {
        d.Dslot = P<int32_t>(q.ep->D->slot);
        d.Dstore = q.prec == SPAMM_F64 ? q.ep->D->store->f64->ptr() : q.ep->D->store->f32->ptr();
      } else {
        // alpha scaling only: an epilogue matrix with no leaves
        d.Dslot = nullptr;
      }
    } else {
      d.alpha = 1.0;
      d.beta = 0.0;
    }
  }
  // placement tables of each launch group: pre[x][k] = units of slice x
  // before request k's part, Q[x] = first unit of slice x (group-relative)
  std::vector<int64_t> sched;
  std::vector<size_t> sched_off;
  const int ns = c->gemm_sched == 1 ? 1 : kXcds;  // slices per request
  for (auto& gk : groups) {
    const auto& rs = gk.second;
    const int nq = int(rs.size());
    sched_off.push_back(sched.size());
    std::vector<int64_t> pre(kXcds * (nq + 1), 0), Q(kXcds + 1, 0);
    for (int x = 0; x < kXcds; ++x) {
      int64_t acc = 0;
      for (int k = 0; k < nq; ++k) {
        const int64_t cn = ht[rs[k]].c_nonnull;
        pre[x * (nq + 1) + k] = acc;
        if (x < ns) acc += cn * (x + 1) / ns - cn * x / ns;
      }
      pre[x * (nq + 1) + nq] = acc;
      Q[x + 1] = Q[x] + acc;
    }
    sched.insert(sched.end(), pre.begin(), pre.end());
    sched.insert(sched.end(), Q.begin(), Q.end());
  }
  // which launch groups run quads
  std::vector<char> gquad;
  for (auto& gk : groups) {
    int64_t kept = 0, leaves = 0;
    for (int r : gk.second) {
      kept += ht[r].n_kept;
      leaves += ht[r].c_nonnull;
    }
    gquad.push_back(quad_group(c, gk.first.first, gk.first.second, kept, leaves));
  }
  // workgroups per launch: the resident maximum, a multiple of 8 (one rank
  // list per XCD)
  std::vector<int> kxs;
  int64_t start_total = 0, scan_need = 0;
  {
    int gi = 0;
    for (auto& gk : groups) {
      const bool quad = gquad[gi];
      const int64_t nwu = launches[gi++].second.second;
      const int64_t maxg = quad ? gemm_quad_max_groups(gk.first.first, c->n_cu)
                                : gemm_max_groups(gk.first.first, gk.first.second, c->gemm_tile, c->n_cu);
      // quads of 64-leaves: at least a quarter of the units (large leaves:
      // one quad per unit)
      const int64_t want =
          std::max<int64_t>(1, std::min<int64_t>(maxg, quad && gk.first.second == 64 ? (nwu + 3) / 4 : nwu));
      const int kx = int((want + kXcds - 1) / kXcds);
      kxs.push_back(kx);
      start_total += int64_t(kXcds) * kx + 1;
      scan_need = std::max<int64_t>(scan_need, int64_t(scan_scratch_bytes(std::max<int64_t>(nwu, 1))));
    }
  }
  RegionP wus, costs, prefix, starts, wn, wt, sscr;
  ALLOC_TMP(wus, std::max<int64_t>(wu_total, 1) * sizeof(WorkUnit), "work units");
  ALLOC_TMP(costs, std::max<int64_t>(wu_total, 1) * 8, "unit costs");
  ALLOC_TMP(prefix, (wu_total + int64_t(groups.size())) * 8, "unit cost prefix");
  ALLOC_TMP(starts, std::max<int64_t>(start_total, 1) * 8, "workgroup ranges");
  ALLOC_TMP(wn, std::max<int64_t>(wu_total, 1) * 8, "unit norms");
  ALLOC_TMP(wt, std::max<int64_t>(wu_total, 1) * 8, "unit diagonal sums");
  ALLOC_TMP(sscr, std::max<int64_t>(scan_need, 1), "scan scratch");
  // quad plans: per quad group, flags, quad positions, step counts and
  // offsets, the quads' cost prefix (int64), the quad records and the steps
  RegionP q_i64, q_rec, q_steps, q_mask, q_pk;
  std::vector<std::array<int64_t, 3>> q_off;  // per group: int64, record and step offsets
  {
    int64_t n64 = 0, nrec = 0, nst = 0, npk = 0;
    std::vector<int64_t> pk_base(count, 0);
    int gi = 0;
    for (auto& gk : groups) {
      const int64_t nwu = launches[gi++].second.second;
      q_off.push_back({n64, nrec, nst});
      if (!gquad[gi - 1]) continue;
      int64_t slots = 0;
      const int bsg = gk.first.second;
      for (int r : gk.second) {
        rd[r].qbase = slots;
        if (bsg == 64) {  // a quad's steps: its products + 1 slots (see k_quad.hip)
          slots += ht[r].n_kept + ht[r].c_nonnull;
          pk_base[r] = npk;
          npk += ht[r].n_kept;
        } else {  // bs / 64 steps per product and 128-tile (four tiles per 256-leaf)
          slots += int64_t(bsg / 64) * (bsg / 128) * (bsg / 128) * ht[r].n_kept;
        }
      }
      n64 += 4 * nwu + 2;
      nrec += nwu;
      nst += slots;
    }
    if (n64 > 0) {
      ALLOC_TMP(q_i64, n64 * 8, "quad plan");
      ALLOC_TMP(q_rec, std::max<int64_t>(nrec, 1) * sizeof(QuadUnit), "quad records");
      ALLOC_TMP(q_steps, std::max<int64_t>(nst, 1) * 16, "quad steps");
      ALLOC_TMP(q_mask, std::max<int64_t>(nst, 1), "quad step children");
      // the k of every kept pair of the quad requests (for the merged k
      // order), at the pair's index
      ALLOC_TMP(q_pk, std::max<int64_t>(npk, 1) * 4, "plan k");
      int gj = 0;
      for (auto& gk : groups) {
        ++gj;
        if (!gquad[gj - 1] || gk.first.second != 64) continue;
        for (int r : gk.second) rd[r].pk = P<int32_t>(q_pk) + pk_base[r];
      }
    }
  }
  // placement tables, the completed request table and C's pyramid jobs:
  // one copy, and the launches after it need no host copies (they may be
  // captured into one graph)
  std::vector<PyrJob> pyr_jobs;
  {
    std::vector<double*> nv;
    std::vector<int> lv;
    for (int r = 0; r < count; ++r) {
      nv.push_back(P<double>(Cs[r]->norms));
      lv.push_back(Cs[r]->L);
    }
    pyr_jobs = pyramid_jobs(nv, lv);
  }
  TableSet postt;
  const size_t o_sched = postt.add(sched), o_req = postt.reserve(count * sizeof(ReqDev)),
               o_pyr = postt.add(pyr_jobs);
  st = place_tables(c, postt);
  if (st != SPAMM_OK) return st;
  {
    int gj = 0;
    for (auto& gk : groups) {
      for (size_t k = 0; k < gk.second.size(); ++k) {
        ReqDev& d = rd[gk.second[k]];
        d.wu_base = launches[gj].second.first;
        d.sched = postt.at<int64_t>(o_sched) + sched_off[gj];
        d.sched_k = int32_t(k);
        d.sched_n = int32_t(gk.second.size());
        d.nslices = ns;
      }
      ++gj;
    }
  }
  postt.put(o_req, rd);
  st = send_tables(c, postt);
  if (st != SPAMM_OK) return st;
  const ReqDev* reqd = postt.at<ReqDev>(o_req);
  const PyrJob* pyr_jd = postt.at<PyrJob>(o_pyr);
  ReqStatsDev* sd_dev = reinterpret_cast<ReqStatsDev*>(c->res_dev + res_tot);
  const ReqStatsDev* sd_host = reinterpret_cast<const ReqStatsDev*>(c->res_host + res_tot);
  auto post = [&]() -> spamm_status {
    {
      TimedScope ts(c, kTPrune);
      SPAMM_HIP(c, launch_prune_fill(c->stream, reqd, count, total_c, cnt_bits, P<int64_t>(scanned),
                                     P<double>(bnd_all), P<int32_t>(cand_all), P<WorkUnit>(wus), P<int64_t>(costs)));
    }
    int gi = 0;
    int64_t soff = 0;
    for (auto& gk : groups) {
      const int64_t u0 = launches[gi].second.first, nwu = launches[gi].second.second;
      const int kx = kxs[gi];
      int64_t* pre = P<int64_t>(prefix) + u0 + gi;
      int64_t* stg = P<int64_t>(starts) + soff;
      soff += int64_t(kXcds) * kx + 1;
      ++gi;
      if (nwu == 0) continue;
      if (gquad[gi - 1]) {
        const auto& qo = q_off[gi - 1];
        int64_t* flag = P<int64_t>(q_i64) + qo[0];
        int64_t* qpos = flag + nwu;        // nwu + 1
        int64_t* qcost = qpos + nwu + 1;   // nwu (zero beyond the last quad)
        int64_t* qpre = qcost + nwu;       // nwu + 1
        QuadUnit* qu = P<QuadUnit>(q_rec) + qo[1];
        int4* steps = P<int4>(q_steps) + qo[2];
        uint8_t* smask = P<uint8_t>(q_mask) + qo[2];
        const WorkUnit* wu = P<WorkUnit>(wus) + u0;
        const int bsg = gk.first.second;
        if (bsg > 64) {  // one quad per unit; flag[0] receives the number of quads
          TimedScope ts(c, kTPrune);
          SPAMM_HIP(c, launch_quad_plan_big(c->stream, reqd, wu, nwu, bsg,
                                            gk.first.first == SPAMM_BF16 || gk.first.first == SPAMM_BF16X3 ? 1 : 0,
                                            qu, qcost, steps, smask, flag));
          SPAMM_HIP(c, launch_scan_i64(c->stream, qcost, qpre, nwu, sscr->ptr(), sscr->bytes));
          SPAMM_HIP(c, launch_wg_ranges(c->stream, qpre, nwu, kXcds * kx, stg));
        } else {
          TimedScope ts(c, kTPrune);
          SPAMM_HIP(c, launch_quad_mark(c->stream, wu, nwu, flag));
          SPAMM_HIP(c, launch_scan_i64(c->stream, flag, qpos, nwu, sscr->ptr(), sscr->bytes));
          SPAMM_HIP(c, launch_zero_i32(c->stream, reinterpret_cast<int32_t*>(qcost), 2 * nwu));
          SPAMM_HIP(c, launch_quad_plan(c->stream, reqd, wu, nwu, flag, qpos, qu, qcost, steps, smask,
                                        gemm_quad_pad_even(gk.first.first) ? 1 : 0));
          SPAMM_HIP(c, launch_scan_i64(c->stream, qcost, qpre, nwu, sscr->ptr(), sscr->bytes));
          SPAMM_HIP(c, launch_wg_ranges(c->stream, qpre, nwu, kXcds * kx, stg));
        }
        GemmArgs ga{};
        ga.wu = wu;
        ga.start = stg;
        ga.reqs = reqd;
        ga.base = c->arena.base();
        ga.wn = P<double>(wn) + u0;
        ga.wt = P<double>(wt) + u0;
        ga.kx = kx;
        ga.interleave = std::max(c->gemm_interleave, 0);  // automatic: contiguous ranges
        ga.qu = qu;
        ga.steps = steps;
        ga.smask = smask;
        ga.nq = bsg > 64 ? flag : qpos + nwu;
        TimedScope ts(c, kTGemm);
        if (c->timing) {
          for (int r : gk.second)
            c->gemm_flops += 2.0 * double(reqs[r].A->bs) * reqs[r].A->bs * reqs[r].A->bs * double(ht[r].n_kept);
          ++c->gemm_quad_launches;
        }
        SPAMM_HIP(c, launch_gemm_quad(c->stream, gk.first.first, bsg, ga));
        continue;
      }
      {
        TimedScope ts(c, kTPrune);
        SPAMM_HIP(c, launch_scan_i64(c->stream, P<int64_t>(costs) + u0, pre, nwu, sscr->ptr(), sscr->bytes));
        SPAMM_HIP(c, launch_wg_ranges(c->stream, pre, nwu, kXcds * kx, stg));
      }
      GemmArgs ga{};
      ga.wu = P<WorkUnit>(wus) + u0;
      ga.start = stg;
      ga.reqs = reqd;
      ga.base = c->arena.base();
      ga.wn = P<double>(wn) + u0;
      ga.wt = P<double>(wt) + u0;
      ga.kx = kx;
      ga.interleave = c->gemm_interleave;
      if (ga.interleave < 0) {
        // short units (few products each): round-robin single units keep an
        // XCD's workgroups close together in its slice; long units: contiguous
        // ranges keep consecutive C leaves (shared A rows) in one workgroup
        int64_t kept = 0;
        for (int r : gk.second) kept += ht[r].n_kept;
        ga.interleave = kept < 16 * nwu ? 1 : 0;
      }
      TimedScope ts(c, kTGemm);
      if (c->timing) {
        for (int r : gk.second)
          c->gemm_flops += 2.0 * double(reqs[r].A->bs) * reqs[r].A->bs * reqs[r].A->bs * double(ht[r].n_kept);
      }
      SPAMM_HIP(c, launch_gemm(c->stream, gk.first.first, gk.first.second, c->gemm_tile, ga));
    }
    {
      TimedScope ts(c, kTPyr);
      SPAMM_HIP(c, launch_unit_scatter(c->stream, reqd, P<WorkUnit>(wus), wu_total, P<double>(wn),
                                       P<double>(wt)));
      if (any_sym) SPAMM_HIP(c, launch_mirror(c->stream, reqd, count, total_c));
    }
    spamm_status s2 = pyramids_launch(c, pyr_jd, pyr_jobs);
    if (s2 != SPAMM_OK) return s2;
    if (st_out) SPAMM_HIP(c, launch_stats_final(c->stream, reqd, count, P<StatPartial>(part), sd_dev));
    return SPAMM_OK;
  };
  if (c->use_graph && !c->timing) {
    // one graph per batch; an instantiated graph of the same shape is
    // updated in place instead of instantiated again
    // recorded on a private stream (the caller's may be the legacy default
    // stream, which cannot be captured) and launched on the caller's
    if (!c->cap_stream) SPAMM_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    SPAMM_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    c->stream = c->cap_stream;
    const spamm_status s1 = post();
    c->stream = user;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (s1 != SPAMM_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return s1 != SPAMM_OK ? s1 : fail(c, SPAMM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (c->gexec) {
      hipGraphNode_t bad = nullptr;
      hipGraphExecUpdateResult res;
      if (hipGraphExecUpdate(c->gexec, g, &bad, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
      }
    }
    hipError_t e2 = hipSuccess;
    if (!c->gexec) e2 = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
      c->gexec = nullptr;
      return fail(c, SPAMM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e2));
    }
    SPAMM_HIP(c, hipGraphLaunch(c->gexec, c->stream));
  } else {
    st = post();
    if (st != SPAMM_OK) return st;
  }

  // ---- statistics (written by the kernel into mapped host memory)
  if (st_out) {
    SPAMM_HIP(c, hipStreamSynchronize(c->stream));
    const std::vector<ReqStatsDev> hs(sd_host, sd_host + count);
    for (int r = 0; r < count; ++r) {
      const spamm_request& q = reqs[r];
      spamm_stats& o = st_out[r];
      std::memset(&o, 0, sizeof(o));
      o.n_kept = ht[r].n_kept;
      o.c_nonnull = ht[r].c_nonnull;
      o.n_candidates = hs[r].n_candidates;
      o.flops = 2.0 * double(q.A->bs) * q.A->bs * q.A->bs * double(ht[r].n_kept);
      o.B1 = q.mode == SPAMM_TRUNCMUL ? 0.0 : hs[r].B1;
      o.B2 = q.mode == SPAMM_TRUNCMUL ? 0.0 : std::sqrt(hs[r].B2sq);
      o.trace = hs[r].trace;
      o.normC = std::sqrt(hs[r].normC_sq);
      o.normA = std::sqrt(hs[r].normA_sq);
      o.normB = std::sqrt(hs[r].normB_sq);
      o.normA_used = std::sqrt(hs[r].normAu_sq);
      o.dA = std::sqrt(hs[r].dA_sq);
      o.dB = std::sqrt(hs[r].dB_sq);
      o.prec_bound = std::sqrt(hs[r].pb_sq);
      if (q.mode == SPAMM_SPAMM || q.mode == SPAMM_SPAMM_SYM) o.err_bound = o.B2;
      else if (q.mode == SPAMM_TRUNCMUL) o.err_bound = o.dA * o.normB + o.normA_used * o.dB;
      else o.err_bound = o.dA * o.normB + o.normA_used * o.dB + o.B2;
    }
  }
  for (int r = 0; r < count; ++r) {
    c->live_handles++;
    C_out[r] = Cs[r].release();
  }
  return SPAMM_OK;
}

spamm_status spamm_multiply(spamm_ctx* ctx, const spamm_mat* A, const spamm_mat* B, double tau, spamm_mode mode,
                            spamm_prec prec, const spamm_epilogue* ep, spamm_mat** C, spamm_stats* st) {
  spamm_request q;
  q.A = A;
  q.B = B;
  q.tau = tau;
  q.mode = mode;
  q.prec = prec;
  q.ep = ep;
  return spamm_multiply_batch(ctx, 1, &q, C, st);
}

spamm_status spamm_norms(spamm_ctx* ctx, const spamm_mat* m, int32_t level, double* out, int64_t cap,
                         int64_t* count) {
  if (!ctx || !m || !count) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (level < -1 || level > m->L) return fail(c, SPAMM_EINVAL, "bad level");
  const int64_t off = level < 0 ? 0 : level_offset(level);
  const int64_t cnt = level < 0 ? pyramid_size(m->L) : (int64_t(1) << (2 * level));
  *count = cnt;
  if (!out || cap < cnt) return fail(c, SPAMM_EINVAL, "output too small");
  return download(c, out, P<double>(m->norms) + off, cnt * 8);
}

spamm_status spamm_kept(spamm_ctx* ctx, const spamm_mat* C, int32_t* ijk, int64_t cap, int64_t* count) {
  if (!ctx || !C || !count) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (!C->plan_off) return fail(c, SPAMM_EINVAL, "handle has no product plan");
  *count = C->n_kept;
  if (!ijk || cap < C->n_kept) return fail(c, SPAMM_EINVAL, "output too small");
  if (C->n_kept == 0) return SPAMM_OK;
  RegionP tmp;
  ALLOC(tmp, C->n_kept * 12, "kept triples");
  SPAMM_HIP(c, launch_decode_kept(c->stream, C->G, P<int64_t>(C->plan_off), P<int2>(C->plan_pairs), C->plan_aoff,
                                  P<int32_t>(C->plan_Astore->keys), P<int32_t>(tmp)));
  return download(c, ijk, tmp->ptr(), C->n_kept * 12);
}

spamm_status spamm_skipped_bound(spamm_ctx* ctx, const spamm_mat* C, double* out, int64_t cap) {
  if (!ctx || !C || !out) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (!C->plan_bnd) return fail(c, SPAMM_EINVAL, "handle has no product plan");
  const int64_t G2 = int64_t(C->G) * C->G;
  if (cap < G2) return fail(c, SPAMM_EINVAL, "output too small");
  return download(c, out, C->plan_bnd->ptr(), G2 * 8);
}

spamm_status spamm_gershgorin(spamm_ctx* ctx, const spamm_mat* m, double* lo, double* hi) {
  if (!ctx || !m || !lo || !hi) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  const Store& s = *m->store;
  if (!s.f64 && !s.f32) return fail(c, SPAMM_EUNSUPPORTED, "no FP64/FP32 leaf copy");
  RegionP part, res;
  ALLOC(part, int64_t(m->G) * 16, "Gershgorin partials");
  ALLOC(res, 16, "Gershgorin bounds");
  SPAMM_HIP(c, launch_gershgorin(c->stream, m->n, m->bs, m->G, P<int32_t>(m->slot), P<double>(s.f64),
                                 s.f64 ? nullptr : P<float>(s.f32), P<double>(part), P<double>(res)));
  double h[2];
  spamm_status st = download(c, h, res->ptr(), 16);
  if (st != SPAMM_OK) return st;
  *lo = h[0];
  *hi = h[1];
  return SPAMM_OK;
}

spamm_status spamm_gershgorin_static(spamm_ctx* ctx, const spamm_mat* m, double* bounds) {
  if (!ctx || !m || !bounds) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (m->ctx != c) return fail(c, SPAMM_EINVAL, "bad matrix handle");
  if (!m->store || (!m->store->f64 && !m->store->f32)) return fail(c, SPAMM_EUNSUPPORTED, "no FP64/FP32 leaf copy");
  if (m->G > kGershStaticRows)
    return fail(c, SPAMM_EUNSUPPORTED, "more leaf rows than the static scratch holds (1024)");
  double* part = noalloc_scratch(c->device);
  if (!part) return fail(c, SPAMM_EDEVICE, "static scratch not set up on this device");
  // every partial in [0, 2 G) is written by the row kernel before the final
  // kernel reads it, so nothing left by an earlier call needs clearing
  const Store& s = *m->store;
  SPAMM_HIP(c, launch_gershgorin(c->stream, m->n, m->bs, m->G, P<int32_t>(m->slot), P<double>(s.f64),
                                 s.f64 ? nullptr : P<float>(s.f32), part, bounds));
  return SPAMM_OK;
}

spamm_status spamm_leaves(spamm_ctx* ctx, const spamm_mat* m, const int32_t* ij, int64_t count, double* out) {
  if (!ctx || !m || (count > 0 && (!ij || !out)) || count < 0) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (count == 0) return SPAMM_OK;
  for (int64_t t = 0; t < count; ++t)
    if (ij[2 * t] < 0 || ij[2 * t] >= m->G || ij[2 * t + 1] < 0 || ij[2 * t + 1] >= m->G)
      return fail(c, SPAMM_EINVAL, "leaf coordinate outside the grid");
  const int64_t e2 = int64_t(m->bs) * m->bs;
  RegionP dij, dout;
  ALLOC(dij, count * 8, "leaf coordinates");
  ALLOC(dout, count * e2 * 8, "gathered leaves");
  spamm_status st = upload(c, dij->ptr(), ij, count * 8);
  if (st != SPAMM_OK) return st;
  const Store& s = *m->store;
  SPAMM_HIP(c, launch_gather_leaves(c->stream, m->bs, count, P<int32_t>(m->slot), P<double>(s.f64),
                                    s.f64 ? nullptr : P<float>(s.f32), P<int32_t>(dij), P<double>(dout)));
  return download(c, out, dout->ptr(), count * e2 * 8);
}

spamm_status spamm_to_dense(spamm_ctx* ctx, const spamm_mat* m, double* out, int64_t ld) {
  if (!ctx || !m || !out) return SPAMM_EINVAL;
  Ctx* c = &ctx->c;
  if (ld < m->n) return fail(c, SPAMM_EINVAL, "ld < n");
  if (!m->store || (!m->store->f64 && !m->store->f32)) return fail(c, SPAMM_EUNSUPPORTED, "no FP64/FP32 copy");
  SPAMM_HIP(c, launch_to_dense(c->stream, m->n, m->bs, m->G, P<int32_t>(m->slot), P<double>(m->store->f64),
                               m->store->f64 ? nullptr : P<float>(m->store->f32), out, ld));
  return SPAMM_OK;
}

spamm_status spamm_mat_info_get(const spamm_mat* m, spamm_mat_info* out) {
  if (!m || !out) return SPAMM_EINVAL;
  out->n = m->n;
  out->leaf = m->bs;
  out->G = m->G;
  out->L = m->L;
  out->nonnull = m->nonnull;
  out->stores = m->store ? m->store->mask() : 0u;
  out->has_plan = m->plan_off ? 1 : 0;
  out->n_kept = m->n_kept;
  out->device_bytes = m->device_bytes();
  return SPAMM_OK;
}

spamm_status spamm_release(spamm_ctx* ctx, spamm_mat* m) {
  if (!m) return SPAMM_OK;
  if (!ctx || m->ctx != &ctx->c) return SPAMM_EINVAL;
  ctx->c.live_handles--;
  delete m;
  return SPAMM_OK;
}

}  // extern "C"
