// Quads of 64-leaves for the leaf GEMM.  The four children of a node of C
// (C leaves (2I + r, 2J + c), r, c in {0, 1}) share their A leaves by row
// half and their B leaves by column half: for a k kept by children (r, 0)
// and (r, 1), one load of A_{2I+r, k} serves both.  A quad is the run of a
// request's work units with one parent (placement keeps a request's C leaves
// in Morton order, so siblings are neighbours); its children's products, each
// list k ascending, are merged into steps in ascending k: a step names the
// A leaves of the two row halves, the B leaves of the two column halves (a
// half no child of the step needs repeats its partner's leaf) and the
// children that keep that k.  Every child still sums its own products k
// ascending, so C does not depend on which siblings share its quad.
//
// The plan: quad starts (flag) and their scan, then one wave per quad marks
// each child's k in an LDS bit set, walks k in chunks of 64 (one lane per
// k) and writes the steps; a child's product index at k is the count of its
// set bits below k (ballot prefix).  A quad's steps are no more than its
// children's products, plus one when the count is padded to even (a step
// no child keeps, for kernels that take two steps per barrier), so they go
// at (its first product's index in the request's list) + (its first C
// leaf's slot in the request), which leaves every quad products + 1 slots
// in Morton order, with no scan; the cost (steps + 1) by quad index feeds
// the workgroup ranges.
#include "internal.h"
#include "kern_common.h"

namespace spamm {

__device__ __forceinline__ uint32_t parent_of(const WorkUnit& w) { return uint32_t(w.cflags & kUnitMorton) >> 2; }

__global__ void k_quad_mark(const WorkUnit* __restrict__ wu, int64_t nwu, int64_t* __restrict__ flag) {
  const int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u >= nwu) return;
  bool start = u == 0;
  if (!start) {
    const WorkUnit w = wu[u], p = wu[u - 1];
    start = p.req != w.req || parent_of(p) != parent_of(w);
  }
  flag[u] = start ? 1 : 0;
}

hipError_t launch_quad_mark(hipStream_t s, const WorkUnit* wu, int64_t nwu, int64_t* flag) {
  if (nwu == 0) return hipSuccess;
  hipLaunchKernelGGL(k_quad_mark, dim3(uint32_t((nwu + 255) / 256)), dim3(256), 0, s, wu, nwu, flag);
  return hipGetLastError();
}

constexpr int kQuadMaxG = 2048;  // leaves per side (the library's largest grid)
constexpr int kQuadWaves = 4;    // quads per workgroup

__global__ void __launch_bounds__(kQuadWaves * 64) k_quad_plan(const ReqDev* __restrict__ reqs,
                                                               const WorkUnit* __restrict__ wu, int64_t nwu,
                                                               const int64_t* __restrict__ flag,
                                                               const int64_t* __restrict__ qpos,
                                                               QuadUnit* __restrict__ qu, int64_t* __restrict__ cost,
                                                               int4* __restrict__ steps, uint8_t* __restrict__ smask,
                                                               int pad_even) {
  __shared__ uint32_t bits[kQuadWaves][4][kQuadMaxG / 32];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t u = int64_t(blockIdx.x) * kQuadWaves + w;
  if (u >= nwu || flag[u] == 0) return;  // wave-uniform; no workgroup barrier below
  const WorkUnit w0 = wu[u];
  const ReqDev& R = reqs[w0.req];
  // the children: units u .. u + n - 1 (the next quad start ends the run)
  int n = 0, cmask = 0;
  int child[4];
  int64_t off[4];
  int32_t cnt[4];
  int32_t kmin = INT32_MAX, kmax = -1;
  bool in = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    in = in && u + i < nwu && (i == 0 || flag[u + i] == 0);
    child[i] = 0;
    off[i] = 0;
    cnt[i] = 0;
    if (in) {
      const WorkUnit x = wu[u + i];
      child[i] = int(x.cflags & kUnitMorton) & 3;
      off[i] = x.pp - R.pairs_idx;  // first product within the request's list
      cnt[i] = x.cnt;
      cmask |= 1 << child[i];
      if (x.cnt > 0) {
        kmin = min(kmin, R.pk[off[i]]);
        kmax = max(kmax, R.pk[off[i] + x.cnt - 1]);
      }
      ++n;
    }
  }
  const int64_t sp = R.qbase + off[0] + (int64_t(w0.cidx) - R.cidx);
  int32_t t = 0;  // steps written
  int4 last = make_int4(-1, -1, -1, -1);  // the last step written
  if (kmax >= 0) {
    uint32_t(*B)[kQuadMaxG / 32] = bits[w];
    const int w0i = (kmin & ~63) >> 5, w1i = (kmax | 63) >> 5;  // words of the chunks walked
#pragma unroll
    for (int i = 0; i < 4; ++i)
      for (int x = w0i + lane; x <= w1i; x += 64) B[i][x] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < 4; ++i)
      for (int j = lane; j < cnt[i]; j += 64) {
        const int32_t k = R.pk[off[i] + j];
        atomicOr(&B[i][k >> 5], 1u << (k & 31));
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int32_t done[4] = {0, 0, 0, 0};  // products of each child before the chunk
    const uint64_t lt = lanemask_lt();
    for (int k0 = kmin & ~63; k0 <= kmax; k0 += 64) {
      const int k = k0 + lane;
      int32_t a[2] = {-1, -1}, b[2] = {-1, -1};
      uint32_t m = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i >= n) break;
        const bool has = (B[i][k >> 5] >> (k & 31)) & 1u;
        const uint64_t bal = ballot64(has);
        if (has) {
          const int2 pr = R.pairs[off[i] + done[i] + popc64(bal & lt)];
          const int c = child[i];
          if (c >> 1) a[1] = pr.x; else a[0] = pr.x;  // A leaf of the row half
          if (c & 1) b[1] = pr.y; else b[0] = pr.y;   // B leaf of the column half
          m |= 1u << c;
        }
        done[i] += popc64(bal);
      }
      const uint64_t any = ballot64(m != 0);
      // a half no child of the step needs takes its partner's leaf (every
      // leaf of a step is then loadable; the children mask says who uses it)
      if (a[0] < 0) a[0] = a[1];
      if (a[1] < 0) a[1] = a[0];
      if (b[0] < 0) b[0] = b[1];
      if (b[1] < 0) b[1] = b[0];
      if (m != 0) {
        const int64_t at = sp + t + popc64(any & lt);
        steps[at] = make_int4(a[0], a[1], b[0], b[1]);
        smask[at] = uint8_t(m);
      }
      if (any) {
        const int hi = 63 - __builtin_clzll(any);  // the lane of the chunk's last step
        last = make_int4(__builtin_amdgcn_readlane(a[0], hi), __builtin_amdgcn_readlane(a[1], hi),
                         __builtin_amdgcn_readlane(b[0], hi), __builtin_amdgcn_readlane(b[1], hi));
      }
      t += popc64(any);
    }
  }
  if (pad_even && (t & 1)) {  // a step no child keeps, over the last step's leaves
    if (lane == 0) {
      steps[sp + t] = last;
      smask[sp + t] = 0;
    }
    ++t;
  }
  if (lane == 0) {
    const int64_t qi = qpos[u];
    QuadUnit r;
    r.sp = sp;
    r.ns = t;
    r.u0 = int32_t(u);
    r.cmask = cmask;
    r.req = w0.req;
    qu[qi] = r;
    cost[qi] = int64_t(t) + 1;
  }
}

// Quads of large leaves (128 and 256): a work unit is a 128 x 128 tile of
// one C leaf, run by the quad kernel as four 64 x 64 children that keep
// every step.  A product A(I,K) B(K,J) of bs = 64 s contributes s steps (its
// k blocks of 64, ascending); a step names the 64 x 64 blocks of A in the
// tile's two block rows and of B in its two block columns, as offsets from
// the arena base in units of 64 elements (A row-major, FP32/FP64 B
// row-major with k as its row, BF16 B from the transposed copy with k
// contiguous).  One wave per unit.  The four tiles of a 256-leaf share their
// leaf's products, so a leaf's steps take 4 s slots per product, tile t at
// s t cnt after the leaf's first: a unit's steps sit at the request's step
// base plus s (tiles * first product + t * cnt), with no scan.
__global__ void __launch_bounds__(256) k_quad_plan_big(const ReqDev* __restrict__ reqs,
                                                       const WorkUnit* __restrict__ wu, int64_t nwu, int bs,
                                                       int bf, QuadUnit* __restrict__ qu, int64_t* __restrict__ cost,
                                                       int4* __restrict__ steps, uint8_t* __restrict__ smask,
                                                       int64_t* __restrict__ nq) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t u = int64_t(blockIdx.x) * 4 + w;
  if (u == 0 && lane == 0) *nq = nwu;
  if (u >= nwu) return;
  const WorkUnit x = wu[u];
  const ReqDev& R = reqs[x.req];
  const int spp = bs / 64;                                 // steps per product
  const int nsub = bs / 128;                               // 128-tiles per side
  const int tile = unit_tile(x.cflags);
  const uint32_t tr = uint32_t((tile / nsub) * 128), tc = uint32_t((tile % nsub) * 128);
  const uint32_t lu = uint32_t(bs) * uint32_t(bs) * (bf ? 2u : 1u) / 64u;  // 64-element units per stored leaf
  const int64_t off = x.pp - R.pairs_idx;                  // first product within the request's list
  const int64_t sp = R.qbase + int64_t(spp) * (int64_t(nsub) * nsub * off + int64_t(tile) * x.cnt);
  const int32_t ns = spp * x.cnt;
  if (lane == 0) {
    QuadUnit q;
    q.sp = sp;
    q.ns = ns;
    q.u0 = int32_t(u);
    q.cmask = 0xF;
    q.req = x.req;
    qu[u] = q;
    cost[u] = int64_t(ns) + 1;
  }
  for (int32_t t = lane; t < ns; t += 64) {
    const int2 pr = R.pairs[off + t / spp];
    const uint32_t kh = uint32_t(t % spp);
    const uint32_t ab = uint32_t(pr.x) * lu, bb = uint32_t(pr.y) * lu;
    const uint32_t a0 = ab + tr * uint32_t(bs) / 64u + kh, a1 = a0 + uint32_t(bs);  // block rows tr, tr + 64
    uint32_t b0, b1;
    if (bf) {  // transposed copy: row j, k contiguous
      b0 = bb + tc * uint32_t(bs) / 64u + kh;
      b1 = b0 + uint32_t(bs);
    } else {  // row k, j contiguous
      b0 = bb + kh * uint32_t(bs) + tc / 64u;
      b1 = b0 + 1u;
    }
    steps[sp + t] = make_int4(int32_t(a0), int32_t(a1), int32_t(b0), int32_t(b1));
    smask[sp + t] = 0xF;
  }
}

hipError_t launch_quad_plan_big(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, int64_t nwu, int bs, int bf,
                                QuadUnit* qu, int64_t* cost, int4* steps, uint8_t* smask, int64_t* nq) {
  if (bs != 128 && bs != 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_quad_plan_big, dim3(uint32_t(std::max<int64_t>((nwu + 3) / 4, 1))), dim3(256), 0, s, reqs,
                     wu, nwu, bs, bf, qu, cost, steps, smask, nq);
  return hipGetLastError();
}

hipError_t launch_quad_plan(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, int64_t nwu, const int64_t* flag,
                            const int64_t* qpos, QuadUnit* qu, int64_t* cost, int4* steps, uint8_t* smask,
                            int pad_even) {
  if (nwu == 0) return hipSuccess;
  hipLaunchKernelGGL(k_quad_plan, dim3(uint32_t((nwu + kQuadWaves - 1) / kQuadWaves)), dim3(kQuadWaves * 64), 0, s,
                     reqs, wu, nwu, flag, qpos, qu, cost, steps, smask, pad_even);
  return hipGetLastError();
}

}  // namespace spamm
