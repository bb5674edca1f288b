// Pruning: which leaf products are formed (Alg. 1's norm test with Alg. 2's
// null rule).  For every C leaf (i, j) one wavefront walks the row i of A and
// the column j of B over the k range where both have non-null leaves, 64 k at
// a time, and keeps k when A_ik and B_kj are non-null and (SpAMM, Hybrid)
// sqrt(s_ik) * sqrt(s_kj) >= tau in FP64.  Because a parent's squared norm is
// a sum of non-negative terms, every ancestor of a kept triple passes the
// same test, so this flat test selects exactly the leaf products reached by
// the recursion of Alg. 1.
//
// Counting pass -> LDS-staged exclusive scan over all C leaves of the batch
// (Morton order) -> fill pass writing the pairs (A and B leaf indices from
// the arena base), the C slot map and the GEMM work units.  No atomics: positions come from the scan, so
// the lists are deterministic.
#include "internal.h"
#include "kern_common.h"

namespace spamm {

constexpr int64_t kCntBits = 40;
constexpr int64_t kCntMask = (int64_t(1) << kCntBits) - 1;

// Requests' first global C index, cached in LDS by every workgroup (larger
// batches search the descriptor table in memory).
constexpr int kReqLds = 512;

__device__ __forceinline__ void cache_cbase(const ReqDev* __restrict__ reqs, int nreq, int64_t* sc) {
  for (int t = threadIdx.x; t < min(nreq, kReqLds); t += blockDim.x) sc[t] = reqs[t].cbase;
  __syncthreads();
}

__device__ __forceinline__ int find_req(const ReqDev* __restrict__ reqs, const int64_t* sc, int nreq, int64_t g) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((nreq <= kReqLds ? sc[mid] : reqs[mid].cbase) <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Each wave takes 64 consecutive C leaves (one per lane).  Every lane finds
// its request, intersects the k ranges of its A row and B column and keeps
// the base addresses of that row and column in the row-major / column-major
// prune views; the wave then walks the leaves whose range is not empty, four
// at a time, 64 k per step, so the loads of four leaves are in flight
// together.
struct LaneLeaf {
  int r;
  uint32_t c, i, j;
  int lo, hi;
  const double* sa;  // sqrt norms of A's row i (index k)
  const double* sb;  // sqrt norms of B's column j
  const int32_t* la;  // slots of A's row i
  const int32_t* lb;  // slots of B's column j
  bool valid;
};

__device__ __forceinline__ LaneLeaf lane_leaf(const ReqDev* __restrict__ reqs, const int64_t* sc, int nreq,
                                              int64_t total_c, int64_t g) {
  LaneLeaf x;
  x.valid = g < total_c;
  x.r = 0;
  x.c = x.i = x.j = 0;
  x.lo = 1;
  x.hi = 0;
  x.sa = x.sb = nullptr;
  x.la = x.lb = nullptr;
  if (x.valid) {
    x.r = find_req(reqs, sc, nreq, g);
    const ReqDev& R = reqs[x.r];
    const int G = R.G;
    x.c = uint32_t(g - R.cbase);
    demorton(x.c, x.i, x.j);
    x.lo = max(R.A.ranges[x.i], R.B.ranges[2 * G + x.j]);
    x.hi = min(R.A.ranges[G + x.i], R.B.ranges[3 * G + x.j]);
    x.sa = R.A.rm_sqrt + int64_t(x.i) * G;
    x.sb = R.B.cm_sqrt + int64_t(x.j) * G;
    x.la = R.A.rm_slot + int64_t(x.i) * G;
    x.lb = R.B.cm_slot + int64_t(x.j) * G;
  }
  return x;
}

__device__ __forceinline__ const double* lane_ptr(const double* p, int b) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(v), b), hi = __builtin_amdgcn_readlane(uint32_t(v >> 32), b);
  return reinterpret_cast<const double*>((uint64_t(hi) << 32) | lo);
}
__device__ __forceinline__ const int32_t* lane_ptr(const int32_t* p, int b) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(v), b), hi = __builtin_amdgcn_readlane(uint32_t(v >> 32), b);
  return reinterpret_cast<const int32_t*>((uint64_t(hi) << 32) | lo);
}

// One walk group: up to four leaves (lanes b[q]), their parameters read from
// those lanes.
struct Group {
  int n;
  int b[4];
  int lo[4], hi[4];
  const double* sa[4];
  const double* sb[4];
  double tau[4];
  bool norms[4];
};

__device__ __forceinline__ Group take_group(uint64_t& todo, const LaneLeaf& x, const ReqDev* __restrict__ reqs) {
  Group gr;
  gr.n = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    gr.b[q] = 0;
    gr.lo[q] = 1;
    gr.hi[q] = 0;
    gr.sa[q] = gr.sb[q] = nullptr;
    gr.tau[q] = 0.0;
    gr.norms[q] = false;
    if (todo) {
      const int b = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1;
      gr.b[q] = b;
      gr.lo[q] = __builtin_amdgcn_readlane(x.lo, b);
      gr.hi[q] = __builtin_amdgcn_readlane(x.hi, b);
      gr.sa[q] = lane_ptr(x.sa, b);
      gr.sb[q] = lane_ptr(x.sb, b);
      const int r = __builtin_amdgcn_readlane(x.r, b);
      gr.tau[q] = reqs[r].tau;
      gr.norms[q] = reqs[r].use_norms != 0;
      gr.n = q + 1;
    }
  }
  return gr;
}

__global__ void __launch_bounds__(256) k_prune_count(const ReqDev* __restrict__ reqs, int nreq, int64_t total_c,
                                                     int64_t* __restrict__ packed, double* __restrict__ bnd_all,
                                                     int32_t* __restrict__ cand_all) {
  __shared__ int64_t sc[kReqLds];
  cache_cbase(reqs, nreq, sc);
  const int64_t g0 = (int64_t(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave;
  if (g0 >= total_c) return;
  const int64_t g = g0 + lane_id();
  const LaneLeaf x = lane_leaf(reqs, sc, nreq, total_c, g);
  int64_t my_cnt = 0, my_cand = 0;
  double my_skip = 0.0;
  uint64_t todo = ballot64(x.valid && x.lo <= x.hi);
  while (todo) {
    const Group gr = take_group(todo, x, reqs);
    int64_t cnt[4] = {0, 0, 0, 0}, cand[4] = {0, 0, 0, 0};
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    int span = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) span = max(span, gr.hi[q] - gr.lo[q] + 1);
    for (int kb = 0; kb < span; kb += kWave) {
      double a[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // all loads first
        const int k = gr.lo[q] + kb + lane_id();
        a[q] = -1.0;
        bv[q] = -1.0;
        if (q < gr.n && k <= gr.hi[q]) {
          a[q] = gr.sa[q][k];
          bv[q] = gr.sb[q][k];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool both = (a[q] >= 0.0) && (bv[q] >= 0.0);
        const double pr = a[q] * bv[q];
        const bool keep = both && (!gr.norms[q] || pr >= gr.tau[q]);
        cnt[q] += popc64(ballot64(keep));
        cand[q] += popc64(ballot64(both));
        if (both && !keep) part[q] += pr;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q >= gr.n) break;
      const double skipped = wave_sum_f64(part[q]);
      if (lane_id() == gr.b[q]) {
        my_cnt = cnt[q];
        my_cand = cand[q];
        my_skip = skipped;
      }
    }
  }
  if (x.valid) {
    const ReqDev& R = reqs[x.r];
    const bool dflag = R.slotD != nullptr && R.slotD[x.c] >= 0;
    const int64_t flag = (my_cnt > 0 || dflag) ? 1 : 0;
    packed[g] = (flag << kCntBits) | my_cnt;
    bnd_all[g] = my_skip;
    cand_all[g] = int32_t(my_cand);
  }
}

hipError_t launch_prune_count(hipStream_t s, const ReqDev* reqs, int nreq, int64_t total_c, int64_t* packed,
                              double* bnd_all, int32_t* cand_all) {
  const int64_t waves = (total_c + kWave - 1) / kWave;
  const int64_t blocks = (waves + 3) / 4;
  hipLaunchKernelGGL(k_prune_count, dim3(uint32_t(blocks)), dim3(256), 0, s, reqs, nreq, total_c, packed,
                     bnd_all, cand_all);
  return hipGetLastError();
}

__global__ void k_gather_totals(const ReqDev* __restrict__ reqs, int nreq, const int64_t* __restrict__ scanned,
                                ReqTotals* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nreq) return;
  const ReqDev& R = reqs[r];
  const int64_t a = scanned[R.cbase], b = scanned[R.cbase + int64_t(R.G) * R.G];
  out[r].n_kept = (b & kCntMask) - (a & kCntMask);
  out[r].c_nonnull = (b >> kCntBits) - (a >> kCntBits);
}

hipError_t launch_gather_totals(hipStream_t s, const ReqDev* reqs, int nreq, const int64_t* scanned,
                                ReqTotals* out) {
  hipLaunchKernelGGL(k_gather_totals, dim3(uint32_t((nreq + 63) / 64)), dim3(64), 0, s, reqs, nreq, scanned, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_prune_fill(const ReqDev* __restrict__ reqs, int nreq, int64_t total_c,
                                                    const int64_t* __restrict__ scanned,
                                                    const double* __restrict__ bnd_all,
                                                    const int32_t* __restrict__ cand_all,
                                                    WorkUnit* __restrict__ wu, int64_t* __restrict__ cost) {
  __shared__ int64_t sc[kReqLds];
  cache_cbase(reqs, nreq, sc);
  const int64_t g0 = (int64_t(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave;
  if (g0 >= total_c) return;
  const int64_t g = g0 + lane_id();
  const LaneLeaf x = lane_leaf(reqs, sc, nreq, total_c, g);
  int64_t off = 0, cnt = 0;
  if (x.valid) {
    const ReqDev& R = reqs[x.r];
    const int64_t G2 = int64_t(R.G) * R.G;
    const int64_t s0 = scanned[R.cbase], sg = scanned[g], s1 = scanned[g + 1];
    off = (sg & kCntMask) - (s0 & kCntMask);
    cnt = (s1 & kCntMask) - (sg & kCntMask);
    const bool flag = ((s1 >> kCntBits) - (sg >> kCntBits)) != 0;
    const int32_t cs = int32_t((sg >> kCntBits) - (s0 >> kCntBits));
    R.off[x.c] = off;
    if (x.c == G2 - 1) R.off[G2] = off + cnt;
    R.cslot[x.c] = flag ? cs : -1;
    R.bnd[x.c] = bnd_all[g];
    R.ncand[x.c] = cand_all[g];
    if (flag) {
      R.ckeys[cs] = int32_t(x.c);
      // placement: slice q of every request's C leaves (Morton order) goes to
      // region q, which the workgroups of XCD q work through
      const int64_t cn = ((scanned[R.cbase + G2] >> kCntBits) - (s0 >> kCntBits));
      const int n = R.sched_n, ns = R.nslices;
      int q = 0;
      while (q + 1 < ns && cn * (q + 1) / ns <= cs) ++q;
      const int64_t* Q = R.sched + kXcds * (n + 1);  // offsets of the slices
      const int64_t at = Q[q] + R.sched[q * (n + 1) + R.sched_k] + (cs - cn * q / ns);
      if (at >= 0 && at < Q[kXcds]) {
        WorkUnit u;
        u.pp = R.pairs_idx + off;
        u.cnt = int32_t(cnt);
        u.cidx = int32_t(R.cidx + cs);
        u.req = x.r;
        u.cflags = int32_t(x.c) | (R.use_ep ? kUnitEp : 0);
        wu[R.wu_base + at] = u;
        cost[R.wu_base + at] = cnt + 1;
      }
    } else {
      R.cnorm[level_offset(R.L) + x.c] = 0.0;
    }
    if (x.i == x.j) R.trace_part[x.i] = 0.0;
  }
  uint64_t todo = ballot64(x.valid && cnt > 0);
  while (todo) {
    const Group gr = take_group(todo, x, reqs);
    int64_t pos[4], end[4];
    const int32_t* la[4];
    const int32_t* lb[4];
    int64_t aoff[4], boff[4];
    int2* out[4];
    int span = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = gr.b[q];
      pos[q] = int64_t((uint64_t(uint32_t(__builtin_amdgcn_readlane(int32_t(uint64_t(off) >> 32), b))) << 32) |
                       uint32_t(__builtin_amdgcn_readlane(int32_t(uint64_t(off)), b)));
      end[q] = pos[q] + __builtin_amdgcn_readlane(int32_t(cnt), b);
      la[q] = lane_ptr(x.la, b);
      lb[q] = lane_ptr(x.lb, b);
      const int r = __builtin_amdgcn_readlane(x.r, b);
      aoff[q] = reqs[r].aoff;
      boff[q] = reqs[r].boff;
      out[q] = reqs[r].pairs;
      if (q < gr.n) span = max(span, gr.hi[q] - gr.lo[q] + 1);
    }
    for (int kb = 0; kb < span; kb += kWave) {
      double a[4], bv[4];
      int32_t sa[4], sb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // norms and slots of four leaves in flight together
        const int k = gr.lo[q] + kb + lane_id();
        a[q] = -1.0;
        bv[q] = -1.0;
        sa[q] = sb[q] = 0;
        if (q < gr.n && k <= gr.hi[q]) {
          a[q] = gr.sa[q][k];
          bv[q] = gr.sb[q][k];
          sa[q] = la[q][k];
          sb[q] = lb[q][k];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool both = (a[q] >= 0.0) && (bv[q] >= 0.0);
        const bool keep = both && (!gr.norms[q] || a[q] * bv[q] >= gr.tau[q]);
        const uint64_t mask = ballot64(keep);
        const int64_t at = pos[q] + popc64(mask & lanemask_lt());
        if (keep && at < end[q]) out[q][at] = make_int2(int32_t(aoff[q] + sa[q]), int32_t(boff[q] + sb[q]));
        pos[q] += popc64(mask);
      }
    }
  }
}

hipError_t launch_prune_fill(hipStream_t s, const ReqDev* reqs, int nreq, int64_t total_c,
                             const int64_t* scanned, const double* bnd_all, const int32_t* cand_all,
                             WorkUnit* wu, int64_t* cost) {
  const int64_t waves = (total_c + kWave - 1) / kWave;
  const int64_t blocks = (waves + 3) / 4;
  hipLaunchKernelGGL(k_prune_fill, dim3(uint32_t(blocks)), dim3(256), 0, s, reqs, nreq, total_c, scanned,
                     bnd_all, cand_all, wu, cost);
  return hipGetLastError();
}

// Per-request accounting, reduced in one fixed order: partial sums over
// chunks of kStatChunk C leaves (one workgroup each), then one workgroup per
// request adds its partials in chunk order with the trace parts and gathers
// the pyramid roots and truncation results, so that one copy brings every
// statistic to the host.
__global__ void __launch_bounds__(256) k_stats_partial(const ReqDev* __restrict__ reqs, int nreq,
                                                       StatPartial* __restrict__ partial) {
  __shared__ double red[4];
  __shared__ int64_t ired[4];
  int lo = 0, hi = nreq - 1;
  const int64_t chunk = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (reqs[mid].stat_base <= chunk) lo = mid;
    else hi = mid - 1;
  }
  const ReqDev& R = reqs[lo];
  const int64_t G2 = int64_t(R.G) * R.G;
  const int64_t c0 = (chunk - R.stat_base) * kStatChunk;
  const int64_t c1 = min<int64_t>(G2, c0 + kStatChunk);
  double b1 = 0.0, b2 = 0.0;
  int64_t cand = 0;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const double b = R.bnd[c];
    b1 += b;
    const double bb = b * b;
    b2 += bb;
    cand += R.ncand[c];
  }
  b1 = block_sum_f64(b1, red);
  b2 = block_sum_f64(b2, red);
  cand = wave_sum_i64(cand);
  __syncthreads();
  if (lane_id() == 0) ired[threadIdx.x / kWave] = cand;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < 4; ++w) t += ired[w];
    partial[chunk].b1 = b1;
    partial[chunk].b2 = b2;
    partial[chunk].cand = t;
  }
}

__global__ void __launch_bounds__(256) k_stats_final(const ReqDev* __restrict__ reqs,
                                                     const StatPartial* __restrict__ partial,
                                                     ReqStatsDev* __restrict__ out) {
  __shared__ double red[4];
  const ReqDev& R = reqs[blockIdx.x];
  const int64_t G2 = int64_t(R.G) * R.G;
  const int64_t nch = (G2 + kStatChunk - 1) / kStatChunk;
  double tr = 0.0;
  for (int64_t i = threadIdx.x; i < R.G; i += blockDim.x) tr += R.trace_part[i];
  tr = block_sum_f64(tr, red);
  if (threadIdx.x == 0) {
    double b1 = 0.0, b2 = 0.0;
    int64_t cand = 0;
    for (int64_t q = 0; q < nch; ++q) {
      b1 += partial[R.stat_base + q].b1;
      b2 += partial[R.stat_base + q].b2;
      cand += partial[R.stat_base + q].cand;
    }
    ReqStatsDev o;
    o.B1 = b1;
    o.B2sq = b2;
    o.trace = tr;
    o.normC_sq = R.cnorm[0];
    o.normA_sq = *R.rootA;
    o.normB_sq = *R.rootB;
    o.normAu_sq = *R.rootAu;
    o.dA_sq = R.truncA ? R.truncA[0] : 0.0;
    o.dB_sq = R.truncB ? R.truncB[0] : 0.0;
    o.n_candidates = cand;
    out[blockIdx.x] = o;
  }
}

hipError_t launch_req_stats(hipStream_t s, const ReqDev* reqs, int nreq, int64_t nchunks, StatPartial* partial,
                            ReqStatsDev* out) {
  if (nreq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats_partial, dim3(uint32_t(nchunks)), dim3(256), 0, s, reqs, nreq, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_final, dim3(uint32_t(nreq)), dim3(256), 0, s, reqs, partial, out);
  return hipGetLastError();
}

// (I, K, J) triples of a product's plan, for parity checks.
__global__ void k_decode_kept(int G, const int64_t* __restrict__ off, const int2* __restrict__ pairs,
                              int64_t aoff, const int32_t* __restrict__ akeys, int32_t* __restrict__ ijk) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= int64_t(G) * G) return;
  uint32_t i, j;
  demorton(uint32_t(c), i, j);
  for (int64_t t = off[c]; t < off[c + 1]; ++t) {
    uint32_t ai, ak;
    demorton(uint32_t(akeys[pairs[t].x - aoff]), ai, ak);
    ijk[3 * t] = int32_t(i);
    ijk[3 * t + 1] = int32_t(ak);
    ijk[3 * t + 2] = int32_t(j);
  }
}

hipError_t launch_decode_kept(hipStream_t s, int G, const int64_t* off, const int2* pairs, int64_t aoff,
                              const int32_t* akeys, int32_t* ijk) {
  const int64_t G2 = int64_t(G) * G;
  hipLaunchKernelGGL(k_decode_kept, dim3(uint32_t((G2 + 255) / 256)), dim3(256), 0, s, G, off, pairs, aoff, akeys,
                     ijk);
  return hipGetLastError();
}

}  // namespace spamm
