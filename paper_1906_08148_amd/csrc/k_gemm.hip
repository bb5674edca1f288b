// Batched leaf products (Sec. 4.4: the output structure is built first, then
// every lowest-level product runs in one batch; Sec. 5.2 counts them as
// 2*bs^3 flops each).
//
// One persistent launch serves every C leaf of every request in a batch.  A
// workgroup pops C leaves from a device queue (the only atomic), and owns the
// whole sum C_ij = sum_k A_ik B_kj: products are streamed in the plan's order
// (k ascending) in k-panels through LDS and accumulated in MFMA registers, so
// results are bitwise reproducible and independent of the batch they run in.
//
// Tiling (wave64, gfx950): the C leaf is split over a 2 x 2 grid of waves
// (one wave for 16 x 16 leaves); each wave holds (BS/2)^2 accumulators as
// 16 x 16 MFMA tiles (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64).  A
// k-panel of A (BS x KP) is staged row-major with a 16-byte row pad; the
// matching panel of B (KP x BS) row-major with an XOR column swizzle so the
// four lane groups of an MFMA operand read different banks.  Lane group g of
// a wave takes the panel's k = g*KP/4 + m, reading four consecutive k of A
// with one 16-byte LDS load.  The next panel is prefetched into registers
// while the current one is multiplied.
//
// The epilogue writes the C leaf, its FP64 squared Frobenius norm (leaf level
// of C's pyramid) and, on diagonal leaves, the diagonal sum for the trace;
// optionally C = alpha * AB + beta * D.
#include <type_traits>

#include "internal.h"
#include "kern_common.h"

namespace spamm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Vec16;
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef double f64x2v __attribute__((ext_vector_type(2)));
template <>
struct Vec16<float> {
  using type = f32x4v;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = f64x2v;
  static constexpr int n = 2;
};

template <typename T, int BS>
struct GemmCfg {
  static constexpr int NW = BS >= 32 ? 4 : 1;
  static constexpr int WM = BS >= 32 ? 2 : 1;
  static constexpr int WN = BS >= 32 ? 2 : 1;
  static constexpr int TILE_M = BS / WM, TILE_N = BS / WN;
  // MFMA tile: 32 x 32 x 2 for FP32 when a wave's tile allows it (the faster
  // FP32 form on gfx950), else 16 x 16 x 4
  static constexpr int MT = (sizeof(T) == 4 && TILE_M % 32 == 0) ? 32 : 16;
  static constexpr int NG = 64 / MT;       // lane groups = k slices of an MFMA
  static constexpr int AE = MT * MT / 64;  // accumulator registers per tile
  static constexpr int TM = TILE_M / MT, TN = TILE_N / MT;
  static constexpr int KP = (BS >= 128 || (sizeof(T) == 8 && BS >= 64)) ? 32 : BS;
  static constexpr int NPANEL = BS / KP;
  static constexpr int NT = NW * 64;
  static constexpr int VN = 16 / int(sizeof(T));
  static constexpr int SA = KP + VN;
  static constexpr int A_VECS = BS * KP / VN / NT;
  static constexpr int B_VECS = KP * BS / VN / NT;
  static constexpr int KG = KP / NG;       // k values of one lane group per panel
  static_assert(A_VECS * VN * NT == BS * KP, "A panel must split evenly");
  static_assert(B_VECS * VN * NT == KP * BS, "B panel must split evenly");
  static_assert(KG % 4 == 0, "lane group takes k in fours");
};

typedef float f32x16 __attribute__((ext_vector_type(16)));

template <typename T, int MT>
struct AccSel {
  using type = typename std::conditional<std::is_same<T, float>::value, f32x4, f64x4>::type;
};
template <>
struct AccSel<float, 32> {
  using type = f32x16;
};
template <typename T, int BS>
using Acc = typename AccSel<T, GemmCfg<T, BS>::MT>::type;

template <typename T, int BS>
__device__ __forceinline__ Acc<T, BS> mfma_step(T a, T b, Acc<T, BS> c) {
  if constexpr (GemmCfg<T, BS>::MT == 32) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  } else if constexpr (std::is_same<T, float>::value) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
}

// Row within an MFMA tile of accumulator register v held by lane group g:
// f32 16x16x4: rows 4g..4g+3; f64 16x16x4: row 4v + g (interleaved);
// f32 32x32x2: row 8(v/4) + 4g + v%4.
template <typename T, int BS>
__device__ __forceinline__ int acc_row(int g, int v) {
  if constexpr (GemmCfg<T, BS>::MT == 32) return 8 * (v / 4) + 4 * g + (v % 4);
  else if constexpr (std::is_same<T, float>::value) return 4 * g + v;
  else return 4 * v + g;
}

// B panel column swizzle: lane group g reads its k rows at column ^ swizzle,
// so the groups of one MFMA operand hit different LDS banks.
template <typename T, int BS>
__device__ __forceinline__ int b_swizzle(int g) {
  return (g * GemmCfg<T, BS>::MT) % BS;
}

template <typename T>
struct WuMeta {
  const ReqDev* R;
  const int2* pairs;
  const T* Ast;
  const T* Bst;
  int64_t pb;
  int64_t np;  // panels
  int32_t c, cslot;
  int32_t cnt;
  int32_t la, lb;  // lane l holds the slots of product pb + 64 * window + l
};

// Fetch the slot pairs of products [pb + base, pb + base + 64) one per lane.
template <typename T>
__device__ __forceinline__ void fetch_pairs(WuMeta<T>& m, int64_t base) {
  const int l = threadIdx.x & 63;
  m.la = 0;
  m.lb = 0;
  if (base + l < m.cnt) {
    const auto pp = as_global(reinterpret_cast<const int32_t*>(m.pairs + m.pb + base + l));
    m.la = pp[0];
    m.lb = pp[1];
  }
}

template <typename T, int BS>
using ARegs = typename Vec16<T>::type[GemmCfg<T, BS>::A_VECS];
template <typename T, int BS>
using BRegs = typename Vec16<T>::type[GemmCfg<T, BS>::B_VECS];

template <typename T, int BS>
__device__ __forceinline__ void load_panel_at(ARegs<T, BS>& ra, BRegs<T, BS>& rb, int32_t sa, int32_t sb, int sub,
                                              const T* __restrict__ Ast, const T* __restrict__ Bst, int tid) {
  using Cf = GemmCfg<T, BS>;
  using V = typename Vec16<T>::type;
  const auto Ag = as_global(Ast + int64_t(sa) * BS * BS + sub * Cf::KP);
  const auto Bg = as_global(Bst + int64_t(sb) * BS * BS + int64_t(sub) * Cf::KP * BS);
#pragma unroll
  for (int t = 0; t < Cf::A_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    const int row = v / (Cf::KP / Cf::VN), cv = v % (Cf::KP / Cf::VN);
    ra[t] = *reinterpret_cast<const __attribute__((address_space(1))) V*>(Ag + int64_t(row) * BS + cv * Cf::VN);
  }
#pragma unroll
  for (int t = 0; t < Cf::B_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    const int kr = v / (BS / Cf::VN), cv = v % (BS / Cf::VN);
    rb[t] = *reinterpret_cast<const __attribute__((address_space(1))) V*>(Bg + int64_t(kr) * BS + cv * Cf::VN);
  }
}

// Panel q of work unit m: product q / NPANEL of the unit, k-panel q % NPANEL.
// The slot pair comes from the lane that holds it (readlane), so no load sits
// between the barrier and the panel's global loads; units with more than 64
// products refill the lane window every 64 products.
template <typename T, int BS>
__device__ __forceinline__ void load_panel(ARegs<T, BS>& ra, BRegs<T, BS>& rb, WuMeta<T>& m, int64_t q, int tid) {
  using Cf = GemmCfg<T, BS>;
  const int64_t p = q / Cf::NPANEL;
  const int sub = int(q % Cf::NPANEL);
  if (p >= 64 && (p & 63) == 0 && sub == 0) fetch_pairs(m, p);
  const int lane = int(p & 63);
  const int32_t sa = __builtin_amdgcn_readlane(m.la, lane);
  const int32_t sb = __builtin_amdgcn_readlane(m.lb, lane);
  load_panel_at<T, BS>(ra, rb, sa, sb, sub, m.Ast, m.Bst, tid);
}

template <typename T, int BS>
__device__ __forceinline__ void store_panel(const ARegs<T, BS>& ra, const BRegs<T, BS>& rb, T* As, T* Bs,
                                            int tid) {
  using Cf = GemmCfg<T, BS>;
  using V = typename Vec16<T>::type;
#pragma unroll
  for (int t = 0; t < Cf::A_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    const int row = v / (Cf::KP / Cf::VN), cv = v % (Cf::KP / Cf::VN);
    *reinterpret_cast<V*>(As + row * Cf::SA + cv * Cf::VN) = ra[t];
  }
#pragma unroll
  for (int t = 0; t < Cf::B_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    const int kr = v / (BS / Cf::VN), cv = v % (BS / Cf::VN);
    const int sw = b_swizzle<T, BS>(kr / Cf::KG);
    *reinterpret_cast<V*>(Bs + kr * BS + ((cv * Cf::VN) ^ sw)) = rb[t];
  }
}

__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

// Wave-uniform description of one work unit (one C leaf).
template <typename T, int BS>
__device__ __forceinline__ WuMeta<T> load_meta(const ReqDev* __restrict__ reqs, const WorkUnit* __restrict__ wus,
                                               int64_t w) {
  WuMeta<T> m;
  const auto ug = as_global(wus + w);
  WorkUnit u;
  u.req = ug->req;
  u.c = ug->c;
  u.pb = ug->pb;
  u.cnt = ug->cnt;
  u.cslot = ug->cslot;
  m.R = reqs + u.req;
  const auto Rg = as_global(m.R);
  m.pairs = Rg->pairs;
  m.Ast = static_cast<const T*>(Rg->Astore);
  m.Bst = static_cast<const T*>(Rg->Bstore);
  m.pb = u.pb;
  m.np = int64_t(u.cnt) * GemmCfg<T, BS>::NPANEL;
  m.c = u.c;
  m.cslot = u.cslot;
  m.cnt = u.cnt;
  fetch_pairs(m, 0);
  return m;
}

// LDS words needed to stage a C leaf for the vectorised epilogue store.
template <typename T, int BS>
struct EpiCfg {
  using Cf = GemmCfg<T, BS>;
  static constexpr int SC = BS + Cf::VN;
  static constexpr int LDS_ELEMS = BS * Cf::SA + Cf::KP * BS;
  static constexpr bool STAGED = BS * SC <= LDS_ELEMS;
};

template <typename T, int BS>
__device__ __forceinline__ void epilogue(const WuMeta<T>& m, Acc<T, BS> (&acc)[GemmCfg<T, BS>::TM][GemmCfg<T, BS>::TN],
                                         T* smem, double* red, int tid, int lane, int wave, int row0, int col0,
                                         int li, int g) {
  using Cf = GemmCfg<T, BS>;
  using Ep = EpiCfg<T, BS>;
  using V = typename Vec16<T>::type;
  const ReqDev* R = m.R;
  const auto Cl = as_global(static_cast<T*>(R->cstore) + int64_t(m.cslot) * BS * BS);
  const T* Dl = nullptr;
  const bool has_ep = R->use_ep != 0;
  if (has_ep && R->Dslot != nullptr) {
    const int32_t ds = R->Dslot[m.c];
    if (ds >= 0) Dl = static_cast<const T*>(R->Dstore) + int64_t(ds) * BS * BS;
  }
  const T alpha = T(R->alpha), beta = T(R->beta);
  uint32_t ci, cj;
  demorton(uint32_t(m.c), ci, cj);
  double nsq = 0.0, tr = 0.0;
  if constexpr (Ep::STAGED) __syncthreads();  // all waves are done reading the panel buffers
#pragma unroll
  for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
    for (int b = 0; b < Cf::TN; ++b)
#pragma unroll
      for (int v = 0; v < Cf::AE; ++v) {
        const int row = row0 + a * Cf::MT + acc_row<T, BS>(g, v);
        const int col = col0 + b * Cf::MT + li;
        T val = acc[a][b][v];
        if (has_ep) {
          const T prod = alpha * val;
          const T dv = Dl ? beta * as_global(Dl)[row * BS + col] : T(0);
          val = prod + dv;
        }
        if constexpr (Ep::STAGED) smem[row * Ep::SC + col] = val;
        else Cl[row * BS + col] = val;
        const double dval = double(val);
        const double sq = dval * dval;
        nsq += sq;
        if (row == col) tr += dval;
      }
  nsq = wave_sum_f64(nsq);
  tr = wave_sum_f64(tr);
  if (lane == 0) {
    red[wave] = nsq;
    red[Cf::NW + wave] = tr;
  }
  __syncthreads();
  if constexpr (Ep::STAGED) {
    constexpr int NV = BS * BS / Cf::VN / Cf::NT;
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int v = tid + t * Cf::NT;
      const int row = v / (BS / Cf::VN), cv = v % (BS / Cf::VN);
      *reinterpret_cast<__attribute__((address_space(1))) V*>(Cl + row * BS + cv * Cf::VN) =
          *reinterpret_cast<const V*>(smem + row * Ep::SC + cv * Cf::VN);
    }
  }
  if (tid == 0) {
    double s = 0.0, t = 0.0;
    for (int x = 0; x < Cf::NW; ++x) {
      s += red[x];
      t += red[Cf::NW + x];
    }
    as_global(R->cnorm)[level_offset(R->L) + m.c] = s;
    if (ci == cj) as_global(R->trace_part)[ci] = t;
  }
}

// Work distribution: each of the kXcd queues serves one XCD (workgroup w
// runs on XCD w % kXcd) and holds, for every request of the launch, the same
// contiguous slice of its C leaves in Morton order, so neighbouring leaves --
// which share A rows and B columns -- meet in one L2.  The units are stored
// queue by queue (queue x owns wu[Q[x] .. Q[x+1])); a workgroup whose queue
// is empty steals from the next queues in turn.
constexpr int kXcd = 8;

__device__ __forceinline__ int64_t pop_unit(int32_t* __restrict__ queues, const int64_t* __restrict__ Q, int& q) {
  for (int tries = 0; tries < kXcd; ++tries) {
    const int64_t idx = atomicAdd(&queues[q], 1);
    const auto Qg = as_global(Q);
    if (idx < Qg[q + 1] - Qg[q]) return Qg[q] + idx;
    q = (q + 1) % kXcd;
  }
  return -1;
}

template <typename T, int BS>
__global__ void __launch_bounds__((GemmCfg<T, BS>::NT))
    k_gemm(const ReqDev* __restrict__ reqs, const WorkUnit* __restrict__ wus, const int64_t* __restrict__ Q,
           int32_t* __restrict__ queues) {
  using Cf = GemmCfg<T, BS>;
  using Ep = EpiCfg<T, BS>;
  using V = typename Vec16<T>::type;
  __shared__ __attribute__((aligned(16))) T smem[Ep::LDS_ELEMS];
  T* const As = smem;
  T* const Bs = smem + BS * Cf::SA;
  __shared__ double red[2 * Cf::NW];
  __shared__ int64_t qsh[2];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / Cf::WN, wc = wave % Cf::WN;
  const int row0 = wr * Cf::TILE_M, col0 = wc * Cf::TILE_N;
  const int li = lane % Cf::MT, g = lane / Cf::MT;
  const int swz = b_swizzle<T, BS>(g);

  // Work units are taken one ahead: while unit `cur` is multiplied, the
  // metadata and first panel of `nxt` are already being loaded.
  int myq = int(blockIdx.x % kXcd);  // used by thread 0 only
  if (tid == 0) {
    qsh[0] = pop_unit(queues, Q, myq);
    qsh[1] = qsh[0] < 0 ? -1 : pop_unit(queues, Q, myq);
  }
  __syncthreads();
  int64_t cur = uniform_i64(qsh[0]), nxt = uniform_i64(qsh[1]);
  if (cur < 0) return;
  WuMeta<T> mc = load_meta<T, BS>(reqs, wus, cur);
  V ra[Cf::A_VECS], rb[Cf::B_VECS];
  if (mc.np > 0) load_panel<T, BS>(ra, rb, mc, 0, tid);

  for (;;) {
    const bool has_next = nxt >= 0;
    WuMeta<T> mn = mc;
    if (has_next) mn = load_meta<T, BS>(reqs, wus, nxt);
    // claim the unit after next now; its index is read at the end of this
    // unit, so no wave waits on the atomic here
    int32_t raw = 0;
    if (tid == 0 && has_next) raw = atomicAdd(&queues[myq], 1);

    Acc<T, BS> acc[Cf::TM][Cf::TN];
#pragma unroll
    for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
      for (int b = 0; b < Cf::TN; ++b) acc[a][b] = Acc<T, BS>{};

    for (int64_t q = 0; q < mc.np; ++q) {
      __syncthreads();
      store_panel<T, BS>(ra, rb, As, Bs, tid);
      __syncthreads();
      if (q + 1 < mc.np) load_panel<T, BS>(ra, rb, mc, q + 1, tid);
      else if (has_next && mn.np > 0) load_panel<T, BS>(ra, rb, mn, 0, tid);
#pragma unroll
      for (int ch = 0; ch < Cf::KG / 4; ++ch) {
        const int kk = g * Cf::KG + 4 * ch;
        T av[Cf::TM][4];
        T bv[Cf::TN][4];
#pragma unroll
        for (int a = 0; a < Cf::TM; ++a) {
          const T* src = As + (row0 + a * Cf::MT + li) * Cf::SA + kk;
          if constexpr (std::is_same<T, float>::value) {
            const f32x4v x = *reinterpret_cast<const f32x4v*>(src);
            av[a][0] = x[0];
            av[a][1] = x[1];
            av[a][2] = x[2];
            av[a][3] = x[3];
          } else {
            const f64x2v x0 = *reinterpret_cast<const f64x2v*>(src);
            const f64x2v x1 = *reinterpret_cast<const f64x2v*>(src + 2);
            av[a][0] = x0[0];
            av[a][1] = x0[1];
            av[a][2] = x1[0];
            av[a][3] = x1[1];
          }
        }
#pragma unroll
        for (int b = 0; b < Cf::TN; ++b) {
          const int col = (col0 + b * Cf::MT + li) ^ swz;
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) bv[b][qq] = Bs[(kk + qq) * BS + col];
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
#pragma unroll
          for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
            for (int b = 0; b < Cf::TN; ++b) acc[a][b] = mfma_step<T, BS>(av[a][qq], bv[b][qq], acc[a][b]);
      }
    }
    if (mc.np == 0 && has_next && mn.np > 0) load_panel<T, BS>(ra, rb, mn, 0, tid);

    epilogue<T, BS>(mc, acc, smem, red, tid, lane, wave, row0, col0, li, g);

    if (!has_next) break;
    if (tid == 0) {
      const auto Qg = as_global(Q);
      int64_t r = int64_t(raw) < Qg[myq + 1] - Qg[myq] ? Qg[myq] + raw : int64_t(-2);
      if (r == -2) {
        myq = (myq + 1) % kXcd;  // this queue is exhausted: steal from the others
        r = pop_unit(queues, Q, myq);
      }
      qsh[1] = r;
    }
    __syncthreads();  // qsh[1] is visible; epilogue LDS reads are done
    cur = nxt;
    nxt = uniform_i64(qsh[1]);
    mc = mn;
  }
}

template <typename T, int BS>
static hipError_t launch_one(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, const int64_t* Q, int64_t nwu,
                             int32_t* queues, int n_cu) {
  using Cf = GemmCfg<T, BS>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gemm<T, BS>, Cf::NT, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t grid = std::min<int64_t>(std::max<int64_t>(nwu, kXcd), int64_t(n_cu) * per_cu);
  hipLaunchKernelGGL((k_gemm<T, BS>), dim3(uint32_t(grid)), dim3(Cf::NT), 0, s, reqs, wu, Q, queues);
  return hipGetLastError();
}

bool gemm_bf16_built();

bool gemm_supported(int prec, int bs) {
  if (prec != SPAMM_F64 && prec != SPAMM_F32 && prec != SPAMM_BF16 && prec != SPAMM_BF16X3) return false;
  if ((prec == SPAMM_BF16 || prec == SPAMM_BF16X3) && !gemm_bf16_built()) return false;
  return bs == 16 || bs == 32 || bs == 64 || bs == 128;
}

hipError_t launch_gemm_bf16(hipStream_t s, int prec, int bs, const ReqDev* reqs, const WorkUnit* wu,
                            const int64_t* Q, int64_t nwu, int32_t* queues, int n_cu);

hipError_t launch_gemm(hipStream_t s, int prec, int bs, const ReqDev* reqs, const WorkUnit* wu, const int64_t* Q,
                       int64_t nwu, int32_t* queues, int n_cu) {
  if (nwu == 0) return hipSuccess;
  if (prec == SPAMM_F32) {
    switch (bs) {
      case 16: return launch_one<float, 16>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 32: return launch_one<float, 32>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 64: return launch_one<float, 64>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 128: return launch_one<float, 128>(s, reqs, wu, Q, nwu, queues, n_cu);
    }
  } else if (prec == SPAMM_F64) {
    switch (bs) {
      case 16: return launch_one<double, 16>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 32: return launch_one<double, 32>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 64: return launch_one<double, 64>(s, reqs, wu, Q, nwu, queues, n_cu);
      case 128: return launch_one<double, 128>(s, reqs, wu, Q, nwu, queues, n_cu);
    }
  } else {
    return launch_gemm_bf16(s, prec, bs, reqs, wu, Q, nwu, queues, n_cu);
  }
  return hipErrorInvalidValue;
}

}  // namespace spamm
