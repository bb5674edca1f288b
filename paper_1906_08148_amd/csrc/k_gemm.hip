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
  static constexpr int TM = TILE_M / 16, TN = TILE_N / 16;
  static constexpr int KP = (BS >= 128 || (sizeof(T) == 8 && BS >= 64)) ? 32 : BS;
  static constexpr int NPANEL = BS / KP;
  static constexpr int NT = NW * 64;
  static constexpr int VN = 16 / int(sizeof(T));
  static constexpr int SA = KP + VN;
  static constexpr int A_VECS = BS * KP / VN / NT;
  static constexpr int B_VECS = KP * BS / VN / NT;
  static constexpr int KG = KP / 4;
  static_assert(A_VECS * VN * NT == BS * KP, "A panel must split evenly");
  static_assert(B_VECS * VN * NT == KP * BS, "B panel must split evenly");
  static_assert(KG % 4 == 0, "lane group takes k in fours");
};

template <typename T>
using Acc = typename std::conditional<std::is_same<T, float>::value, f32x4, f64x4>::type;

template <typename T>
__device__ __forceinline__ Acc<T> mfma16(T a, T b, Acc<T> c) {
  if constexpr (std::is_same<T, float>::value) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
}

template <typename T, int BS>
__device__ __forceinline__ int b_swizzle(int g) {
  return (g * 16) % BS;
}

template <typename T, int BS>
using ARegs = typename Vec16<T>::type[GemmCfg<T, BS>::A_VECS];
template <typename T, int BS>
using BRegs = typename Vec16<T>::type[GemmCfg<T, BS>::B_VECS];

template <typename T, int BS>
__device__ __forceinline__ void load_panel(ARegs<T, BS>& ra, BRegs<T, BS>& rb,
                                           const int2* __restrict__ pairs, const T* __restrict__ Ast,
                                           const T* __restrict__ Bst, int64_t pb, int64_t q, int tid) {
  using Cf = GemmCfg<T, BS>;
  using V = typename Vec16<T>::type;
  const int64_t p = pb + q / Cf::NPANEL;
  const int sub = int(q % Cf::NPANEL);
  const int2 pr = pairs[p];
  const T* Ag = Ast + int64_t(pr.x) * BS * BS + sub * Cf::KP;
  const T* Bg = Bst + int64_t(pr.y) * BS * BS + int64_t(sub) * Cf::KP * BS;
#pragma unroll
  for (int t = 0; t < Cf::A_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    const int row = v / (Cf::KP / Cf::VN), cv = v % (Cf::KP / Cf::VN);
    ra[t] = *reinterpret_cast<const V*>(Ag + int64_t(row) * BS + cv * Cf::VN);
  }
#pragma unroll
  for (int t = 0; t < Cf::B_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    const int kr = v / (BS / Cf::VN), cv = v % (BS / Cf::VN);
    rb[t] = *reinterpret_cast<const V*>(Bg + int64_t(kr) * BS + cv * Cf::VN);
  }
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

template <typename T, int BS>
__global__ void __launch_bounds__((GemmCfg<T, BS>::NT)) k_gemm(const ReqDev* __restrict__ reqs,
                                                              const WorkUnit* __restrict__ wus, int64_t wu0,
                                                              int64_t nwu, int32_t* __restrict__ queue) {
  using Cf = GemmCfg<T, BS>;
  using V = typename Vec16<T>::type;
  __shared__ __attribute__((aligned(16))) T As[BS * Cf::SA];
  __shared__ __attribute__((aligned(16))) T Bs[Cf::KP * BS];
  __shared__ double red[2 * Cf::NW];
  __shared__ int wu_sh;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / Cf::WN, wc = wave % Cf::WN;
  const int row0 = wr * Cf::TILE_M, col0 = wc * Cf::TILE_N;
  const int li = lane & 15, g = lane >> 4;
  const int swz = b_swizzle<T, BS>(g);

  for (;;) {
    if (tid == 0) wu_sh = atomicAdd(queue, 1);
    __syncthreads();
    const int64_t w = wu_sh;
    __syncthreads();
    if (w >= nwu) break;

    const WorkUnit u = wus[wu0 + w];
    const ReqDev* R = reqs + u.req;
    const int64_t pb = R->off[u.c], pe = R->off[u.c + 1];
    const int2* __restrict__ pairs = R->pairs;
    const T* __restrict__ Ast = static_cast<const T*>(R->Astore);
    const T* __restrict__ Bst = static_cast<const T*>(R->Bstore);
    const int64_t npanel = (pe - pb) * Cf::NPANEL;

    Acc<T> acc[Cf::TM][Cf::TN];
#pragma unroll
    for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
      for (int b = 0; b < Cf::TN; ++b) acc[a][b] = Acc<T>{0, 0, 0, 0};

    V ra[Cf::A_VECS], rb[Cf::B_VECS];
    if (npanel > 0) load_panel<T, BS>(ra, rb, pairs, Ast, Bst, pb, 0, tid);
    for (int64_t q = 0; q < npanel; ++q) {
      __syncthreads();
      store_panel<T, BS>(ra, rb, As, Bs, tid);
      __syncthreads();
      if (q + 1 < npanel) load_panel<T, BS>(ra, rb, pairs, Ast, Bst, pb, q + 1, tid);
#pragma unroll
      for (int ch = 0; ch < Cf::KG / 4; ++ch) {
        const int kk = g * Cf::KG + 4 * ch;
        T av[Cf::TM][4];
        T bv[Cf::TN][4];
#pragma unroll
        for (int a = 0; a < Cf::TM; ++a) {
          const T* src = As + (row0 + a * 16 + li) * Cf::SA + kk;
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
          const int col = (col0 + b * 16 + li) ^ swz;
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) bv[b][qq] = Bs[(kk + qq) * BS + col];
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
#pragma unroll
          for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
            for (int b = 0; b < Cf::TN; ++b) acc[a][b] = mfma16<T>(av[a][qq], bv[b][qq], acc[a][b]);
      }
    }

    // epilogue
    const int32_t cs = R->cslot[u.c];
    T* __restrict__ Cl = static_cast<T*>(R->cstore) + int64_t(cs) * BS * BS;
    const T* __restrict__ Dl = nullptr;
    if (R->Dslot != nullptr) {
      const int32_t ds = R->Dslot[u.c];
      if (ds >= 0) Dl = static_cast<const T*>(R->Dstore) + int64_t(ds) * BS * BS;
    }
    const bool has_ep = R->use_ep != 0;
    const T alpha = T(R->alpha), beta = T(R->beta);
    uint32_t ci, cj;
    demorton(uint32_t(u.c), ci, cj);
    double nsq = 0.0, tr = 0.0;
#pragma unroll
    for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
      for (int b = 0; b < Cf::TN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // accumulator layout: f32 16x16x4 holds rows 4g..4g+3 of column li;
          // f64 16x16x4 interleaves them, register v holding row 4v + g
          const int row = row0 + a * 16 + (std::is_same<T, float>::value ? 4 * g + v : 4 * v + g);
          const int col = col0 + b * 16 + li;
          T val = acc[a][b][v];
          if (has_ep) {
            const T prod = alpha * val;
            const T dv = Dl ? beta * Dl[row * BS + col] : T(0);
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
      red[wave] = nsq;
      red[Cf::NW + wave] = tr;
    }
    __syncthreads();
    if (tid == 0) {
      double s = 0.0, t = 0.0;
      for (int x = 0; x < Cf::NW; ++x) {
        s += red[x];
        t += red[Cf::NW + x];
      }
      R->cnorm[level_offset(R->L) + u.c] = s;
      if (ci == cj) R->trace_part[ci] = t;
    }
  }
}

template <typename T, int BS>
static hipError_t launch_one(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, int64_t wu0, int64_t nwu,
                             int32_t* queue, int n_cu) {
  using Cf = GemmCfg<T, BS>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gemm<T, BS>, Cf::NT, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t grid = std::min<int64_t>(nwu, int64_t(n_cu) * per_cu);
  hipLaunchKernelGGL((k_gemm<T, BS>), dim3(uint32_t(grid)), dim3(Cf::NT), 0, s, reqs, wu, wu0, nwu, queue);
  return hipGetLastError();
}

bool gemm_bf16_built();

bool gemm_supported(int prec, int bs) {
  if (prec != SPAMM_F64 && prec != SPAMM_F32 && prec != SPAMM_BF16 && prec != SPAMM_BF16X3) return false;
  if ((prec == SPAMM_BF16 || prec == SPAMM_BF16X3) && !gemm_bf16_built()) return false;
  return bs == 16 || bs == 32 || bs == 64 || bs == 128;
}

hipError_t launch_gemm_bf16(hipStream_t s, int prec, int bs, const ReqDev* reqs, const WorkUnit* wu, int64_t wu0,
                            int64_t nwu, int32_t* queue, int n_cu);

hipError_t launch_gemm(hipStream_t s, int prec, int bs, const ReqDev* reqs, const WorkUnit* wu, int64_t wu0,
                       int64_t nwu, int32_t* queue, int n_cu) {
  if (nwu == 0) return hipSuccess;
  if (prec == SPAMM_F32) {
    switch (bs) {
      case 16: return launch_one<float, 16>(s, reqs, wu, wu0, nwu, queue, n_cu);
      case 32: return launch_one<float, 32>(s, reqs, wu, wu0, nwu, queue, n_cu);
      case 64: return launch_one<float, 64>(s, reqs, wu, wu0, nwu, queue, n_cu);
      case 128: return launch_one<float, 128>(s, reqs, wu, wu0, nwu, queue, n_cu);
    }
  } else if (prec == SPAMM_F64) {
    switch (bs) {
      case 16: return launch_one<double, 16>(s, reqs, wu, wu0, nwu, queue, n_cu);
      case 32: return launch_one<double, 32>(s, reqs, wu, wu0, nwu, queue, n_cu);
      case 64: return launch_one<double, 64>(s, reqs, wu, wu0, nwu, queue, n_cu);
      case 128: return launch_one<double, 128>(s, reqs, wu, wu0, nwu, queue, n_cu);
    }
  } else {
    return launch_gemm_bf16(s, prec, bs, reqs, wu, wu0, nwu, queue, n_cu);
  }
  return hipErrorInvalidValue;
}

}  // namespace spamm
