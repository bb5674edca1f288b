// Leaf products with one wave per C leaf (leaf sizes 16, 32, 64).
//
// A wave owns a whole C leaf: its BS x BS accumulators are (BS/16)^2 tiles of
// 16 x 16 MFMA accumulators (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64).
// Operand fragments go straight from global memory (L2) into registers in
// MFMA order -- no LDS and no workgroup barriers.  The products of a leaf
// are streamed in the plan's order (k ascending) as "chunks": chunk ch of a
// product covers, for lane group g (lanes 16g..16g+15), the k values
// g*BS/4 + 4ch .. +3, read as four consecutive A entries of the lane's row
// (one 16-byte load) and four B entries of its column.  NB chunks are in
// flight at any time; the stream runs across product and work-unit
// boundaries, so the next C leaf's first operands are already loaded when
// the current one is written.  Work units come from the per-XCD queues one
// unit ahead, and the unit after that is claimed with an atomic whose result
// is only read at the next unit boundary.
//
// Sums are per C leaf in a fixed order (chunks in k order, MFMA order within
// a chunk), so results are bitwise reproducible and equal to the LDS kernel's
// order of products (the sum within one 16x16x4 step is the MFMA's own).
#include <type_traits>

#include "internal.h"
#include "kern_common.h"

namespace spamm {

typedef float wf32x4 __attribute__((ext_vector_type(4)));
typedef double wf64x4 __attribute__((ext_vector_type(4)));
typedef float wf32x4v __attribute__((ext_vector_type(4)));
typedef double wf64x2v __attribute__((ext_vector_type(2)));

template <typename T>
using WAcc = typename std::conditional<std::is_same<T, float>::value, wf32x4, wf64x4>::type;

template <typename T>
__device__ __forceinline__ WAcc<T> wmfma(T a, T b, WAcc<T> c) {
  if constexpr (std::is_same<T, float>::value) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
}

template <typename T, int BS>
struct WCfg {
  static constexpr int TT = BS / 16;  // tiles per side
  static constexpr int KG = BS / 4;   // k values per lane group per product
  static constexpr int CPP = KG / 4;  // chunks per product
  // chunks in flight: exactly one product, so products start at ring slot 0
  // and the window never reaches past the next unit (every unit in the
  // stream has at least one product)
  static constexpr int NB = CPP;
};

template <typename T, int BS>
struct Frag {
  T a[WCfg<T, BS>::TT][4];
  T b[WCfg<T, BS>::TT][4];
};

template <typename T>
struct WMeta {
  const ReqDev* R;
  const int2* pairs;
  const T* Ast;
  const T* Bst;
  int64_t pb;
  int32_t cnt, c, cslot;
  int32_t la, lb;  // lane l: slots of product 64 * window + l
};

__device__ __forceinline__ int64_t wuniform(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

// Claim a unit: lane 0 takes the next index of queue q (stealing from the
// following queues when it is empty); every lane gets the result.
__device__ __forceinline__ int64_t wpop(int32_t* __restrict__ queues, const int64_t* __restrict__ Q, int& q) {
  int64_t r = -1;
  if ((threadIdx.x & 63) == 0) {
    const auto Qg = as_global(Q);
    for (int tries = 0; tries < 8; ++tries) {
      const int64_t idx = atomicAdd(&queues[q], 1);
      if (idx < Qg[q + 1] - Qg[q]) {
        r = Qg[q] + idx;
        break;
      }
      q = (q + 1) % 8;
    }
  }
  q = __shfl(q, 0, 64);
  return wuniform(__shfl(r, 0, 64));
}

// Deferred claim: lane 0 fires the atomic now; the index is read one unit
// later (wresolve), so the wave never waits on the atomic in the fast path.
__device__ __forceinline__ int32_t wclaim(int32_t* __restrict__ queues, int q) {
  int32_t raw = 0;
  if ((threadIdx.x & 63) == 0) raw = atomicAdd(&queues[q], 1);
  return raw;
}

__device__ __forceinline__ int64_t wresolve(int32_t raw, int32_t* __restrict__ queues, const int64_t* __restrict__ Q,
                                            int& q) {
  const int64_t idx = wuniform(__shfl(int64_t(raw), 0, 64));
  const auto Qg = as_global(Q);
  const int64_t lo = Qg[q], hi = Qg[q + 1];
  if (idx < hi - lo) return lo + idx;
  q = (q + 1) % 8;
  return wpop(queues, Q, q);  // this queue is exhausted: steal from the others
}

template <typename T>
__device__ __forceinline__ void wfetch_pairs(WMeta<T>& m, int64_t base) {
  const int l = threadIdx.x & 63;
  m.la = 0;
  m.lb = 0;
  if (base + l < m.cnt) {
    const auto pp = as_global(reinterpret_cast<const int32_t*>(m.pairs + m.pb + base + l));
    m.la = pp[0];
    m.lb = pp[1];
  }
}

template <typename T>
__device__ __forceinline__ WMeta<T> wmeta(const ReqDev* __restrict__ reqs, const WorkUnit* __restrict__ wus,
                                          int64_t w) {
  WMeta<T> m;
  const auto ug = as_global(wus + w);
  const int32_t req = ug->req;
  m.c = ug->c;
  m.pb = ug->pb;
  m.cnt = ug->cnt;
  m.cslot = ug->cslot;
  m.R = reqs + req;
  const auto Rg = as_global(m.R);
  m.pairs = Rg->pairs;
  m.Ast = static_cast<const T*>(Rg->Astore);
  m.Bst = static_cast<const T*>(Rg->Bstore);
  wfetch_pairs(m, 0);
  return m;
}

// Load chunk ch of product p of unit m into f.
template <typename T, int BS>
__device__ __forceinline__ void wload(Frag<T, BS>& f, WMeta<T>& m, int64_t p, int ch) {
  using C = WCfg<T, BS>;
  if (p >= 64 && (p & 63) == 0 && ch == 0) wfetch_pairs(m, p);
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int src = int(p & 63);
  const int32_t sa = __builtin_amdgcn_readlane(m.la, src);
  const int32_t sb = __builtin_amdgcn_readlane(m.lb, src);
  const int k0 = g * C::KG + 4 * ch;
  const auto Ag = as_global(m.Ast + int64_t(sa) * BS * BS);
  const auto Bg = as_global(m.Bst + int64_t(sb) * BS * BS);
#pragma unroll
  for (int a = 0; a < C::TT; ++a) {
    const auto src_a = Ag + (a * 16 + li) * BS + k0;
    if constexpr (std::is_same<T, float>::value) {
      const wf32x4v x = *reinterpret_cast<const __attribute__((address_space(1))) wf32x4v*>(src_a);
      f.a[a][0] = x[0];
      f.a[a][1] = x[1];
      f.a[a][2] = x[2];
      f.a[a][3] = x[3];
    } else {
      const wf64x2v x0 = *reinterpret_cast<const __attribute__((address_space(1))) wf64x2v*>(src_a);
      const wf64x2v x1 = *reinterpret_cast<const __attribute__((address_space(1))) wf64x2v*>(src_a + 2);
      f.a[a][0] = x0[0];
      f.a[a][1] = x0[1];
      f.a[a][2] = x1[0];
      f.a[a][3] = x1[1];
    }
  }
#pragma unroll
  for (int b = 0; b < C::TT; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) f.b[b][q] = Bg[(k0 + q) * BS + b * 16 + li];
}

template <typename T, int BS>
__device__ __forceinline__ void wcompute(const Frag<T, BS>& f, WAcc<T> (&acc)[WCfg<T, BS>::TT][WCfg<T, BS>::TT]) {
  using C = WCfg<T, BS>;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int a = 0; a < C::TT; ++a)
#pragma unroll
      for (int b = 0; b < C::TT; ++b) acc[a][b] = wmfma<T>(f.a[a][q], f.b[b][q], acc[a][b]);
}

// Write the C leaf (optionally alpha * AB + beta * D), its FP64 squared norm
// and, on diagonal leaves, its diagonal sum.  acc may be all zero (a unit
// with no products that exists because D has a leaf there).
template <typename T, int BS, bool ZERO>
__device__ __forceinline__ void wepilogue_impl(const WMeta<T>& m, const WAcc<T>* acc) {
  using C = WCfg<T, BS>;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const auto R = as_global(m.R);
  const auto Cl = as_global(static_cast<T*>(R->cstore) + int64_t(m.cslot) * BS * BS);
  const bool has_ep = R->use_ep != 0;
  const T* Dl = nullptr;
  if (has_ep && R->Dslot != nullptr) {
    const int32_t ds = as_global(R->Dslot)[m.c];
    if (ds >= 0) Dl = static_cast<const T*>(R->Dstore) + int64_t(ds) * BS * BS;
  }
  const T alpha = T(R->alpha), beta = T(R->beta);
  uint32_t ci, cj;
  demorton(uint32_t(m.c), ci, cj);
  double nsq = 0.0, tr = 0.0;
#pragma unroll
  for (int a = 0; a < C::TT; ++a)
#pragma unroll
    for (int b = 0; b < C::TT; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f32 16x16x4 holds rows 4g..4g+3 of column li; f64 interleaves
        // them, register v holding row 4v + g
        const int row = a * 16 + (std::is_same<T, float>::value ? 4 * g + v : 4 * v + g);
        const int col = b * 16 + li;
        T val = ZERO ? T(0) : acc[a * C::TT + b][v];
        if (has_ep) {
          const T prod = alpha * val;
          const T dv = Dl ? beta * as_global(Dl)[row * BS + col] : T(0);
          val = prod + dv;
        }
        Cl[row * BS + col] = val;
        const double dval = double(val);
        const double sq = dval * dval;
        nsq += sq;
        if (row == col) tr += dval;
      }
  nsq = wave_sum_f64(nsq);
  tr = wave_sum_f64(tr);
  if (lane == 0) {
    as_global(R->cnorm)[level_offset(R->L) + m.c] = nsq;
    if (ci == cj) as_global(R->trace_part)[ci] = tr;
  }
}

template <typename T, int BS>
__device__ __forceinline__ void wepilogue(const WMeta<T>& m, const WAcc<T> (&acc)[WCfg<T, BS>::TT][WCfg<T, BS>::TT]) {
  wepilogue_impl<T, BS, false>(m, &acc[0][0]);
}

template <typename T, int BS>
__device__ __attribute__((noinline)) void wepilogue_zero(const WMeta<T> m) {
  wepilogue_impl<T, BS, true>(m, nullptr);
}

template <typename T, int BS>
__global__ void __launch_bounds__(64) k_gemm_wave(const ReqDev* __restrict__ reqs, const WorkUnit* __restrict__ wus,
                                                  const int64_t* __restrict__ Q, int32_t* __restrict__ queues) {
  using C = WCfg<T, BS>;
  constexpr int NB = C::NB;
  WAcc<T> acc[C::TT][C::TT];
#pragma unroll
  for (int a = 0; a < C::TT; ++a)
#pragma unroll
    for (int b = 0; b < C::TT; ++b) acc[a][b] = WAcc<T>{0, 0, 0, 0};

  int myq = int(blockIdx.x % 8);
  // Load unit idx (or the first later one with products); a unit with no
  // products only carries an epilogue and is finished at once.
  auto settle = [&](int64_t idx, WMeta<T>& m) -> bool {
    for (;;) {
      if (idx < 0) return false;
      m = wmeta<T>(reqs, wus, idx);
      if (m.cnt > 0) return true;
      wepilogue_zero<T, BS>(m);
      idx = wpop(queues, Q, myq);
    }
  };
  auto take = [&](int64_t& idx, WMeta<T>& m) -> bool { return settle(idx = wpop(queues, Q, myq), m); };

  int64_t icur, inxt;
  WMeta<T> mc, mn;
  if (!take(icur, mc)) return;
  bool has_next = take(inxt, mn);
  int32_t raw = wclaim(queues, myq);  // the unit after next, read at the next boundary

  // Ring of NB chunk buffers; slot s always holds chunk s % CPP of some
  // product.  mi is the unit being issued: the current one or, once that is
  // fully issued, the next one.
  Frag<T, BS> buf[NB];
  WMeta<T> mi = mc;
  bool mi_is_next = false;
  int64_t ip = 0;
  bool issue_done = false;
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    if (!issue_done) {
      wload<T, BS>(buf[s], mi, ip, s % C::CPP);
      if (s % C::CPP == C::CPP - 1 && ++ip == mi.cnt) {
        ip = 0;
        if (!mi_is_next && has_next) {
          mi = mn;
          mi_is_next = true;
        } else {
          issue_done = true;
        }
      }
    }
  }

  int64_t cp = 0;
  bool finished = false;
  while (!finished) {
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      if (!finished) {
        wcompute<T, BS>(buf[s], acc);
        if (s % C::CPP == C::CPP - 1 && ++cp == mc.cnt) {
          wepilogue<T, BS>(mc, acc);
#pragma unroll
          for (int a = 0; a < C::TT; ++a)
#pragma unroll
            for (int b = 0; b < C::TT; ++b) acc[a][b] = WAcc<T>{0, 0, 0, 0};
          cp = 0;
          if (!has_next) {
            finished = true;
          } else {
            // the issue position already lies in the new current unit
            mc = mn;
            icur = inxt;
            mi_is_next = false;
            inxt = wresolve(raw, queues, Q, myq);
            has_next = settle(inxt, mn);
            raw = wclaim(queues, myq);
            if (issue_done && has_next) {
              mi = mn;
              mi_is_next = true;
              ip = 0;
              issue_done = false;
            }
          }
        }
        if (!finished && !issue_done) {
          wload<T, BS>(buf[s], mi, ip, s % C::CPP);
          if (s % C::CPP == C::CPP - 1 && ++ip == mi.cnt) {
            ip = 0;
            if (!mi_is_next && has_next) {
              mi = mn;
              mi_is_next = true;
            } else {
              issue_done = true;
            }
          }
        }
      }
    }
  }
}

template <typename T, int BS>
static hipError_t wlaunch(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, const int64_t* Q, int64_t nwu,
                          int32_t* queues, int n_cu) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gemm_wave<T, BS>, 64, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t grid = std::min<int64_t>(std::max<int64_t>(nwu, 8), int64_t(n_cu) * per_cu);
  hipLaunchKernelGGL((k_gemm_wave<T, BS>), dim3(uint32_t(grid)), dim3(64), 0, s, reqs, wu, Q, queues);
  return hipGetLastError();
}

bool gemm_wave_supported(int prec, int bs) {
  if (prec == SPAMM_F32) return bs == 16 || bs == 32 || bs == 64;
  if (prec == SPAMM_F64) return bs == 16 || bs == 32;  // leaf 64 in FP64 does not fit one wave
  return false;
}

hipError_t launch_gemm_wave(hipStream_t s, int prec, int bs, const ReqDev* reqs, const WorkUnit* wu, const int64_t* Q,
                            int64_t nwu, int32_t* queues, int n_cu) {
  if (nwu == 0) return hipSuccess;
  if (prec == SPAMM_F32) {
    switch (bs) {
      case 16: return wlaunch<float, 16>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 32: return wlaunch<float, 32>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 64: return wlaunch<float, 64>(s, reqs, wu, Q, nwu, queues, n_cu);
    }
  } else if (prec == SPAMM_F64) {
    switch (bs) {
      case 16: return wlaunch<double, 16>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 32: return wlaunch<double, 32>(s, reqs, wu, Q, nwu, queues, n_cu);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace spamm
