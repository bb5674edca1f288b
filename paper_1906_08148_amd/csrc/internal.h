// Internal declarations of the spamm library (host side and kernel launchers).
// Everything here is private to libspamm.so; the public ABI is include/spamm.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/spamm.h"

namespace spamm {

// ---------------------------------------------------------------- arena

// Sub-allocator over one caller-owned device buffer: first-fit free ranges
// in an ordered map, coalesced on release, with an exact-size cache in
// front: a released range waits in the bucket of its (size, alignment) and
// the next request of that shape takes it back in O(1) (the multiply and
// build calls repeat their shapes from batch to batch).  The buckets return
// to the coalescing range map when a request finds no fit, and before the
// largest free range is reported.  All reuse is ordered on the context's
// single stream.
class Arena {
 public:
  void init(char* base, size_t bytes);
  // Returns offset or SIZE_MAX when no range fits.  high: a short-lived
  // block, from the top of the highest range that fits (last fit).
  size_t alloc(size_t bytes, size_t align = 256, bool high = false);
  // merge: straight back into the range map (short-lived blocks), else into
  // the exact-size cache.
  void release(size_t off, size_t bytes, size_t align, bool merge = false);
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  size_t free_bytes() const { return size_ - used_; }
  size_t largest_free() const;
  char* base() const { return base_; }

 private:
  size_t fit(size_t bytes, size_t align) const;       // first fit in the range map
  size_t fit_high(size_t bytes, size_t align) const;  // last fit in the range map
  void insert_free(size_t off, size_t bytes) const;   // into the range map, merged
  void trim() const;                              // buckets back into the range map
  char* base_ = nullptr;
  size_t size_ = 0;
  size_t used_ = 0;
  mutable std::map<size_t, size_t> free_;  // offset -> length
  mutable std::unordered_map<uint64_t, std::vector<size_t>> cache_;  // (size, log2 align) -> offsets
};

struct Ctx;

// One arena allocation; freed when the last shared owner drops it.
struct Region {
  Ctx* ctx = nullptr;
  size_t off = 0, bytes = 0, align = 256;
  bool temp = false;  // short-lived (see Arena::alloc)
  ~Region();
  void* ptr() const;
};
using RegionP = std::shared_ptr<Region>;

// Leaf storage shared by a matrix and the matrices derived from it.
struct Store {
  int64_t nleaf = 0;  // slots in the store
  int32_t bs = 0;
  RegionP keys;       // int32[nleaf]: Morton key of each stored leaf
  // f64 / f32: leaf s at s * bs^2, row-major.  bf16: leaf s holds the hi
  // parts (bf16 of the FP32 value) then the lo parts (bf16 of the FP32
  // remainder), bs^2 each, row-major; bf16t holds the same two blocks
  // transposed (the B operand of a BF16 product reads its k index
  // contiguously).  Every copy is aligned to its leaf size within the arena,
  // so a leaf is addressed by one index from the arena base.
  RegionP f64, f32, bf16, bf16t;
  uint32_t mask() const {
    return (f64 ? SPAMM_STORE_F64 : 0u) | (f32 ? SPAMM_STORE_F32 : 0u) | (bf16 ? SPAMM_STORE_BF16 : 0u);
  }
};
using StoreP = std::shared_ptr<Store>;

}  // namespace spamm

// The public opaque types.
struct spamm_mat {
  spamm::Ctx* ctx = nullptr;
  int64_t n = 0;
  int32_t bs = 0, G = 0, L = 0;
  int64_t nonnull = -1;     // -1: not read back yet
  spamm::StoreP store;
  spamm::RegionP slot;      // int32[G*G]  Morton -> slot, -1 null
  spamm::RegionP norms;     // double[(4^(L+1)-1)/3], level l at (4^l-1)/3
  spamm::RegionP rm_sqrt;   // double[G*G] row-major sqrt(norm), -1 null
  spamm::RegionP rm_slot;   // int32[G*G]  row-major slot
  spamm::RegionP cm_sqrt;   // double[G*G] [c*G + r] = leaf (r, c)
  spamm::RegionP cm_slot;   // int32[G*G]
  spamm::RegionP ranges;    // int32[4*G]: row_lo, row_hi, col_lo, col_hi
  // set on products only
  spamm::RegionP plan_off;  // int64[G*G+1] local offsets into plan_pairs
  spamm::RegionP plan_pairs;// int2[n_kept]  A and B leaf indices from the arena base
  spamm::RegionP plan_bnd;  // double[G*G] skipped bound b per C leaf
  spamm::StoreP plan_Astore, plan_Bstore;  // keys decode k from the A index
  int64_t plan_aoff = 0;    // A store's first leaf index from the arena base
  int64_t n_kept = -1;
  size_t device_bytes() const;
};

namespace spamm {

enum TimeClass { kTBuild = 0, kTTrunc, kTPrune, kTGemm, kTPyr, kTClasses };

struct Ctx {
  int device = 0;
  // event timing per kernel class
  bool timing = false;
  struct Pending {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  double t_ms[kTClasses] = {0, 0, 0, 0, 0};
  int64_t t_cnt[kTClasses] = {0, 0, 0, 0, 0};
  double gemm_flops = 0.0;
  int64_t gemm_quad_launches = 0;  // timed GEMM launches on quads
  hipEvent_t get_event();
  hipError_t collect_timing();  // sync + fold pending pairs into totals
  hipStream_t stream = nullptr;
  Arena arena;
  std::string last_error;
  // pinned host staging for read-backs
  void* host_stage = nullptr;
  size_t host_stage_bytes = 0;
  // pinned upload ring: each upload takes the next region; a region is
  // reused only after the copy that read it has completed (its event), so
  // uploads do not wait for the stream to drain
  struct UpRec {
    size_t s, e;
    hipEvent_t ev;
  };
  char* up_ring = nullptr;
  size_t up_bytes = 0, up_head = 0;
  std::deque<UpRec> up_inflight;
  std::vector<hipEvent_t> up_events;
  int n_cu = 256;
  int gemm_sched = 0;  // work-unit placement: 0 per-XCD Morton slices, 1 request-major
  int gemm_tile = 1;   // GEMM variant (MFMA tile shape), see launch_gemm
  int gemm_interleave = -1;  // GemmArgs::interleave (chunk of consecutive units, 0: contiguous ranges,
                             // -1: per launch, 1 for short units and 0 for long ones)
  int use_graph = 0;   // launch the post-sizing kernels of a batch as one captured graph
  int validate = 0;    // measure every lower-precision product against an FP64 twin
  int gemm_quad = -1;  // leaf-64 products in quads of sibling C leaves (k_gemm_quad): 1, 0, -1 automatic
  hipGraphExec_t gexec = nullptr;  // last instantiated batch graph (updated in place when the shape repeats)
  hipStream_t cap_stream = nullptr;  // private stream the batch graph is recorded on (nothing runs on it)
  std::map<uint64_t, int> tuned;  // reserved for autotune results
  int live_handles = 0;
  // results that kernels write straight into host memory (mapped pinned,
  // coherent): read by the host after a stream synchronisation
  char* res_host = nullptr;
  char* res_dev = nullptr;
  size_t res_bytes = 0;
  RegionP alloc(size_t bytes, size_t align = 256, bool temp = false);  // nullptr on exhaustion
  void* stage(size_t bytes);      // grow pinned staging if needed
  bool results(size_t bytes);     // res_* holds at least `bytes` (synchronises to grow)
};

// Records events around the launches of one kernel class while timing is on.
struct TimedScope {
  Ctx* c;
  int cls;
  hipEvent_t a = nullptr;
  TimedScope(Ctx* ctx, int k) : c(ctx), cls(k) {
    if (c->timing) {
      a = c->get_event();
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~TimedScope() {
    if (a) {
      hipEvent_t b = c->get_event();
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->pending.push_back({cls, a, b});
      }
    }
  }
};

// status helpers
spamm_status fail(Ctx* c, spamm_status s, const std::string& msg);
#define SPAMM_HIP(ctx, expr)                                                   \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      return ::spamm::fail((ctx), SPAMM_EDEVICE,                               \
                           std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

__host__ __device__ inline int64_t level_offset(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; }
__host__ __device__ inline int64_t pyramid_size(int L) { return level_offset(L + 1); }

// ---------------------------------------------------------------- device descs

// One matrix as seen by the batched kernels.
struct MatDev {
  const int32_t* slot;     // Morton
  const double* leafnorm;  // Morton, leaf level
  const double* rm_sqrt;
  const int32_t* rm_slot;
  const double* cm_sqrt;
  const int32_t* cm_slot;
  const int32_t* ranges;
  int32_t G, L;
};

// Pyramid job: reduce leaf norms (level L) of one matrix up to the root.
struct PyrJob {
  double* norms;  // full pyramid buffer
  int32_t L;
  int32_t sub_levels;   // levels reduced inside one subtree workgroup
  int64_t block_base;   // first workgroup index of this job
  int32_t nsub;         // subtree workgroups of this job
  int32_t pad_;
};

// One multiply request inside a batch.
struct ReqDev {
  MatDev A, B;
  const int32_t* slotD;  // epilogue matrix slot map (Morton) or nullptr
  double tau;
  int32_t use_norms;
  int32_t G, L, bs;
  int64_t cbase;          // first global C index of this request
  // outputs (set after sizing)
  int2* pairs;            // A and B leaf indices from the arena base
  int64_t* off;           // G*G+1 local offsets
  int32_t* cslot;         // C slot map (Morton)
  int32_t* ckeys;         // C keys [c_nonnull]
  double* cnorm;          // C pyramid buffer (leaf level written by GEMM)
  double* bnd;            // skipped bound per C leaf
  int32_t* ncand;         // candidate count per C leaf
  double* trace_part;     // G entries (diagonal leaves)
  void* cstore;           // C leaf store (FP32 or FP64)
  // GEMM operands in the request's precision: first leaf of A's and B's
  // store as an index from the arena base (in leaves of the operand copy)
  int64_t aoff, boff;
  int64_t pairs_idx;      // pairs as an index from the arena base (8-byte units)
  int64_t cidx;           // C store's first leaf as an index from the arena base
  const void* Dstore;
  const int32_t* Dslot;
  double alpha, beta;
  int64_t wu_base;        // first work unit of this request's launch group
  int32_t prec;
  int32_t use_ep;         // apply alpha/beta/D in the epilogue
  // accounting inputs (roots of the pyramids, truncation results)
  const double* rootA;
  const double* rootB;
  const double* rootAu;
  const double* truncA;   // nullptr when A was not truncated
  const double* truncB;
  int64_t stat_base;      // first statistics chunk of this request
  // Work-unit placement: this request's group table (pre[8 * (n + 1)], then
  // the offsets Q[9] of the 8 slices) and its index k in the group
  const int64_t* sched;
  int32_t sched_k, sched_n;
  int32_t nslices;        // slices per request in the placement (8 per-XCD, or 1)
  int32_t sym;            // symmetric square: C leaves below the diagonal are mirrored
  const int32_t* asym;    // symmetric square: nonzero when the operand's (or D's) null
                          // map is not symmetric (every C leaf is then formed)
  int32_t* pk;            // k of every kept pair (nullptr: not needed), beside `pairs`
  int64_t qbase;          // quads: the request's first step slot in its group's step array
};

// One truncation inside a batch (leaf-block truncation with budget tau^2).
struct TruncJob {
  const int32_t* slot;     // input slot map (Morton)
  const double* leafnorm;  // input leaf norms (Morton)
  int32_t* out_slot;
  double* out_norm;        // leaf level of the output pyramid
  double* result;          // [0] dropped squared norm, [1] non-null leaves dropped
  double tau2;
  int64_t base;            // first element in the batch's concatenated arrays
  int32_t G;
  int32_t key_bits_lo;     // bits of the Morton index in the sort key
  int32_t pairs;           // truncate in mirror pairs (I, K) + (K, I), keyed by the upper leaf
};

// Row/column views of one matrix (see ensure_prep).
struct PrepJob {
  const int32_t* slot;
  const double* leafnorm;
  double* rm_sqrt;
  int32_t* rm_slot;
  double* cm_sqrt;
  int32_t* cm_slot;
  int32_t* ranges;
  int64_t base;   // first element (G*G per job)
  int64_t wbase;  // first wave of the range pass (2*G per job)
  int32_t G;
  int32_t pad_;
};

// One C leaf for the GEMM (24 bytes).
struct WorkUnit {
  int64_t pp;      // first product's pair, as an index from the arena base (8-byte units)
  int32_t cnt;     // products (0: the leaf comes from the epilogue matrix alone)
  int32_t cidx;    // C leaf as an index from the arena base (C leaves)
  int32_t req;     // request
  int32_t cflags;  // Morton index of the C leaf | kUnitEp when the epilogue applies alpha/beta/D
};
constexpr int32_t kUnitEp = int32_t(1) << 30;
// Bits 28-29 of cflags: the unit's tile of a C leaf split into tiles (256
// leaves: 2 x 2 tiles of 128, tile = 2 * tile row + tile column); the
// Morton index sits below bit 28, so G <= 16384.
constexpr int kUnitTileShift = 28;
constexpr int32_t kUnitMorton = (int32_t(1) << kUnitTileShift) - 1;
__host__ __device__ inline int unit_tile(int32_t cflags) { return (cflags >> kUnitTileShift) & 3; }

// A quad: the non-null C leaves of one parent node of one request (up to
// four siblings, consecutive work units), run by one workgroup with one wave
// per child over the merged k order of the children's products, so that an
// A leaf serves both children of its row and a B leaf both of its column.
struct QuadUnit {
  int64_t sp;      // first merged step (index into the step arrays)
  int32_t ns;      // merged steps
  int32_t u0;      // first work unit of the quad (launch-group relative)
  int32_t cmask;   // bit c: child c (2 * row half + column half) is present
  int32_t req;     // request
};
static_assert(sizeof(QuadUnit) == 24, "a quad record is three 8-byte words");

// Arguments of one GEMM launch: the work units of one (precision, leaf size)
// group in placement order, split into contiguous ranges of equal cost, one
// per workgroup.
struct GemmArgs {
  const WorkUnit* wu;
  const int64_t* start;  // [nwg + 1]: range of workgroup rank r is [start[r], start[r+1])
  const ReqDev* reqs;
  const char* base;      // arena base
  double* wn;            // per unit: FP64 squared Frobenius norm of the C leaf
  double* wt;            // per unit: diagonal sum of the C leaf (diagonal leaves)
  int32_t kx;            // workgroups per XCD (the grid is 8 * kx)
  int32_t interleave;    // c > 0: an XCD's units [start[x*kx], start[(x+1)*kx]) dealt round-robin over its
                         // workgroups in chunks of c; 0: workgroup rank r takes [start[r], start[r+1])
  // quad launches: the quads, and per merged step the A leaves of the two
  // row halves and the B leaves of the two column halves (a half no child
  // needs repeats its partner's) and the children that take part (bit c)
  const QuadUnit* qu;
  const int4* steps;
  const uint8_t* smask;
  const int64_t* nq;     // number of quads (device)
};

// Per-request totals read back after the counting pass.
struct ReqTotals {
  int64_t n_kept;
  int64_t c_nonnull;
};

// Per-request statistics reduced on the device.
struct ReqStatsDev {
  double B1, B2sq, trace, normC_sq;
  double normA_sq, normB_sq, normAu_sq, dA_sq, dB_sq;
  double pb_sq;  // squared rounding bound of the kept products
  int64_t n_candidates;
};

constexpr int kStatChunk = 4096;  // C leaves per partial-statistics workgroup

// Validation of one product against its FP64 twin: both C stores hold the
// same non-null leaves in the same slots (same kept products).
struct ValJob {
  const float* c32;   // the product's C store (FP32)
  const double* c64;  // the twin's C store (FP64)
  int64_t nelem;      // non-null leaves x bs^2
  int64_t chunk_base; // first chunk of this job in the partial sums
};
constexpr int64_t kValChunk = 65536;  // elements per partial sum

struct StatPartial {
  double b1, b2, pb;
  int64_t cand;
};

// ---------------------------------------------------------------- launchers
// (all enqueue on `s`; return hipError_t of the launch)

hipError_t launch_build_scan_dense(hipStream_t s, const double* dense, int64_t n, int64_t ld,
                                   int bs, int G, double* leafnorm, int32_t* flag,
                                   int32_t* nonfinite);
// One block list of a batched build (device table).  G*G entries and
// blocks are numbered through the batch.  A list's leaf store has one slot
// per listed block (block t -> slot t); slots of all-zero or rejected
// blocks stay unused.
struct BuildJob {
  int64_t n;
  int32_t bs, G;
  int64_t nblocks;
  const int32_t* coords;
  const double* data;
  int32_t* src_of;    // G*G: index of the block placed at each Morton slot
  double* leafnorm;   // leaf level of the norm pyramid
  int32_t* slot;      // slot map
  int32_t* keys;      // Morton key of each leaf slot
  int32_t* err;       // four error words
  int64_t* total;     // non-null leaves
  double* f64;        // leaf copies (null when not kept)
  float* f32;
  uint16_t* b16;
  uint16_t* b16t;
  int64_t g2_base;    // first G*G entry of this list in the batch
  int64_t blk_base;   // first block of this list in the batch
};
// init, scatter, then one pass over the blocks (norms, null flags, slot
// map, keys, leaf copies, counts): one launch each for all lists
hipError_t launch_build_batch(hipStream_t s, const BuildJob* jobs, int njobs, int64_t g2_total,
                              int64_t blocks_total);
// exclusive scan of int32 flags -> slot map (flag ? prefix : -1) and its
// inverse keys[slot] = index (keys may be null), total -> *total
hipError_t launch_flags_to_slots(hipStream_t s, const int32_t* flag, int64_t count, int32_t* slot,
                                 int32_t* keys, int64_t* total, void* scratch, size_t scratch_bytes);
size_t scan_scratch_bytes(int64_t count);
hipError_t launch_scan_i64(hipStream_t s, const int64_t* in, int64_t* out, int64_t count,
                           void* scratch, size_t scratch_bytes);  // exclusive, out[count] = total
hipError_t launch_copy_dense_leaves(hipStream_t s, const double* dense, int64_t n, int64_t ld,
                                    int bs, int64_t nleaf, const int32_t* keys, double* f64,
                                    float* f32, uint16_t* b16, uint16_t* b16t);
hipError_t launch_derive_store(hipStream_t s, int64_t nleaf, int bs, const double* f64, const float* f32,
                               double* o64, float* o32, uint16_t* o16, uint16_t* o16t);
hipError_t launch_prep_batch(hipStream_t s, const PrepJob* jobs_dev, int njobs, int64_t total,
                             int64_t total_waves);
hipError_t launch_pyramid(hipStream_t s, const PyrJob* jobs_dev, int njobs,
                          const std::vector<PyrJob>& jobs_host);
// truncation of several matrices at once (total = sum of G*G)
hipError_t launch_trunc_batch(hipStream_t s, const TruncJob* jobs_dev, int njobs, int64_t total,
                              void* scratch, size_t scratch_bytes);
size_t trunc_batch_scratch_bytes(int njobs, int64_t total);
// prune.  The counting pass packs (C leaf non-null << cnt_bits) | kept count
// per C leaf into one int64, so that one scan gives both prefixes; the host
// picks cnt_bits per batch so that neither field can overflow.
hipError_t launch_prune_count(hipStream_t s, const ReqDev* reqs, int nreq, int64_t total_c, int cnt_bits,
                              int64_t* packed, double* bnd_all, int32_t* cand_all, double* pb_all);
hipError_t launch_gather_totals(hipStream_t s, const ReqDev* reqs, int nreq, int cnt_bits,
                                const int64_t* scanned, ReqTotals* out);
// writes the kept pairs, C's slot map and the work units (with their cost,
// products + 1, for the range split) in placement order
hipError_t launch_prune_fill(hipStream_t s, const ReqDev* reqs, int nreq, int64_t total_c, int cnt_bits,
                             const int64_t* scanned, const double* bnd_all,
                             const int32_t* cand_all, WorkUnit* wu, int64_t* cost);
constexpr int kXcds = 8;  // slices of the placement: workgroup w runs on XCD w % 8
// start[r] = first unit whose cost prefix reaches r / nwg of the total
hipError_t launch_wg_ranges(hipStream_t s, const int64_t* prefix, int64_t nwu, int nwg, int64_t* start);
// GEMM over the work units of one (precision, leaf size) group
// variant 0: 32 x 32 MFMA tiles for FP32 / BF16 where a wave's tile allows
// it; variant 1: 16 x 16 tiles
hipError_t launch_gemm(hipStream_t s, int prec, int bs, int variant, const GemmArgs& a);
// Quads of 64-leaves (see QuadUnit): the quad kernel, its occupancy, and the
// plan: quad starts, then per quad its record, merged steps and cost
// (steps + 1, by quad index).
bool gemm_quad_supported(int prec, int bs);
int gemm_quad_max_groups(int prec, int n_cu);
hipError_t launch_gemm_quad(hipStream_t s, int prec, int bs, const GemmArgs& a);
hipError_t launch_quad_mark(hipStream_t s, const WorkUnit* wu, int64_t nwu, int64_t* flag);
hipError_t launch_quad_plan(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, int64_t nwu, const int64_t* flag,
                            const int64_t* qpos, QuadUnit* qu, int64_t* cost, int4* steps, uint8_t* smask,
                            int pad_even);
bool gemm_quad_pad_even(int prec);  // quad steps padded to an even count
// quads of leaves 128 / 256: one per work unit (a 128 x 128 tile), every
// child kept; *nq receives the number of quads
hipError_t launch_quad_plan_big(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, int64_t nwu, int bs, int bf,
                                QuadUnit* qu, int64_t* cost, int4* steps, uint8_t* smask, int64_t* nq);
int gemm_max_groups(int prec, int bs, int variant, int n_cu);  // resident workgroups of the kernel
bool gemm_supported(int prec, int bs);
int gemm_unit_tiles(int bs);  // work units per C leaf (4 for 256 leaves, else 1)
// leaf norms and trace parts of the units into each request's C pyramid
hipError_t launch_unit_scatter(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, int64_t nwu,
                               const double* wn, const double* wt);
hipError_t launch_zero_i32(hipStream_t s, int32_t* p, int64_t count);
// The entry point that allocates nothing keeps its scratch in a static
// device array of this many leaf rows (noalloc.hip); noalloc_setup looks up
// the array's address on `device` (which must be current) once, and
// noalloc_scratch returns it (nullptr before setup).
constexpr int kGershStaticRows = 1024;
hipError_t noalloc_setup(int device);
double* noalloc_scratch(int device);

hipError_t launch_gershgorin(hipStream_t s, int64_t n, int bs, int G, const int32_t* slot, const double* f64,
                             const float* f32, double* part, double* out);
hipError_t launch_gather_leaves(hipStream_t s, int bs, int64_t count, const int32_t* slot, const double* f64,
                                const float* f32, const int32_t* ij, double* out);
hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t count, int32_t value);
// Element-wise truncation of one matrix into a new store with the same slots.
struct ElemTruncJob {
  int G, bs;
  double tau;
  const int32_t* in_slot;
  const double* in_f64;
  int32_t* slot;      // new slot map (G*G)
  double* leafnorm;   // new leaf level of the pyramid (G*G)
  double* dropped;    // squared norm of the dropped entries per leaf (G*G)
  int64_t* count;     // non-null leaves of the result (starts at zero)
  double* f64;
  float* f32;
  uint16_t* b16;
  uint16_t* b16t;
};
hipError_t launch_trunc_elem(hipStream_t s, const ElemTruncJob& job);
// *out = v[0] + ... + v[n-1] in a fixed order (partial: (n + 4095) / 4096)
hipError_t launch_sum_f64(hipStream_t s, const double* v, int64_t n, double* partial, double* out);
// Symmetric squares: every C leaf below the diagonal of a request with sym
// set becomes the transpose of its mirror, with the mirror's norm.
hipError_t launch_mirror(hipStream_t s, const ReqDev* reqs, int nreq, int64_t total_c);
// flag |= 1 if the null map of slot (or of slotD, nullable) is not symmetric;
// the flag must be zero before
hipError_t launch_sym_check(hipStream_t s, int G, const int32_t* slot, const int32_t* slotD, int32_t* flag);
hipError_t launch_stats_partial(hipStream_t s, const ReqDev* reqs, int nreq, int64_t nchunks,
                                const double* bnd_all, const int32_t* cand_all, const double* pb_all,
                                StatPartial* partial);
hipError_t launch_stats_final(hipStream_t s, const ReqDev* reqs, int nreq, const StatPartial* partial,
                              ReqStatsDev* out);
// out[j] = ||c32 - c64||_F^2 of job j (partial: one double per chunk)
hipError_t launch_validate(hipStream_t s, const ValJob* jobs, int njobs, int64_t nchunks, double* partial,
                           double* out);
hipError_t launch_to_dense(hipStream_t s, int64_t n, int bs, int G, const int32_t* slot,
                           const double* f64, const float* f32, double* out, int64_t ld);
hipError_t launch_decode_kept(hipStream_t s, int G, const int64_t* off, const int2* pairs, int64_t aoff,
                              const int32_t* akeys, int32_t* ijk);

}  // namespace spamm
