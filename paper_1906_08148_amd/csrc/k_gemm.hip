// Batched leaf products (Sec. 4.4: the output structure is built first, then
// every lowest-level product runs in one batch; Sec. 5.3 counts them as
// 2*bs^3 flops each).
//
// One persistent launch serves every C leaf of every request of a batch that
// shares a precision and leaf size.  The work units (one per C leaf) sit in
// placement order -- eight slices, each a Morton-contiguous part of every
// request, so that the leaves one XCD works on share A rows and B columns in
// its L2 -- and are split into contiguous ranges of equal cost (products + 1),
// one per workgroup.  Workgroup w runs on XCD w % 8 and takes the range of
// rank (w % 8) * kx + w / 8, so the ranks of an XCD cover its slice.  There
// are no atomics: a workgroup owns the whole sum C_ij = sum_k A_ik B_kj of
// each of its leaves, streamed in the plan's order (k ascending) through LDS
// in k-panels and accumulated in MFMA registers, so results are bitwise
// reproducible and independent of the batch they run in.
//
// Nothing in the inner loop waits on a dependent load: the unit records of
// the range are held one per lane, 64 units per block (two blocks); the slot
// pairs of the products are held one per lane, 64 per window, three windows
// ahead; the next panel is loaded into registers while the current one is
// multiplied, across unit boundaries too.  Pairs are leaf indices from the
// arena base, so a product's operands need no request descriptor.
//
// Tiling (wave64, gfx950): the C leaf is split over a 2 x 2 grid of waves
// (one wave for 16 x 16 leaves).  MFMA tiles: v_mfma_f64_16x16x4f64 (FP64),
// v_mfma_f32_16x16x4f32 (FP32, variant 1) or 32x32x2f32 (variant 0, where a
// wave's tile is 32 wide), v_mfma_f32_16x16x32_bf16 / 32x32x16_bf16 (BF16,
// the same two variants; split-BF16 takes three
// products per step, lo*hi + hi*lo + hi*hi, in FP32).  A k-panel of A (BS x KP)
// is staged row-major with a 16-byte row pad.  For FP32/FP64 the k-panel of
// B (KP x BS) is row-major with an XOR column swizzle so the lane groups of
// an MFMA operand read different banks; for BF16 the B panel comes from the
// transposed copy (k contiguous per column) and is laid out like A, so each
// lane reads its eight k values with one 16-byte LDS load.
//
// The epilogue writes the C leaf (FP64 for FP64 products, else FP32), the
// leaf's FP64 squared Frobenius norm and, on diagonal leaves, its diagonal
// sum, per unit; optionally C = alpha * AB + beta * D.
//
// Leaves of 256 (LS) are stored row-major like every other leaf size; their
// C leaf is split into 2 x 2 tiles of 128 (BS), one work unit each, so the
// 128-tile kernel runs them with a row stride of 256 and k running over all
// 256 columns of A (and rows of B) of a product.
#include <type_traits>

#include "internal.h"
#include "kern_common.h"

namespace spamm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));

template <int P, int BS, int V, int LS = BS>
struct GemmCfg {
  static constexpr bool kBf = P == SPAMM_BF16 || P == SPAMM_BF16X3;
  static constexpr int NH = P == SPAMM_BF16X3 ? 2 : 1;  // hi / lo halves staged
  static constexpr int ES = P == SPAMM_F64 ? 8 : P == SPAMM_F32 ? 4 : 2;
  using Out = typename std::conditional<P == SPAMM_F64, double, float>::type;
  static constexpr int NW = BS >= 32 ? 4 : 1;
  static constexpr int WM = BS >= 32 ? 2 : 1;
  static constexpr int WN = BS >= 32 ? 2 : 1;
  static constexpr int TILE_M = BS / WM, TILE_N = BS / WN;
  // MFMA tile: 32 x 32 for FP32 / BF16 where a wave's tile allows it
  // (variant 0), else 16 x 16 (variant 1, and always for FP64)
  static constexpr int MT = (V == 0 && P != SPAMM_F64 && TILE_M % 32 == 0) ? 32 : 16;
  static constexpr int NG = 64 / MT;      // lane groups
  static constexpr int AE = MT * MT / 64;  // accumulator registers per tile
  static constexpr int TM = TILE_M / MT, TN = TILE_N / MT;
  static constexpr int KP = P == SPAMM_F64    ? (BS >= 64 ? 32 : BS)
                            : P == SPAMM_F32  ? (BS >= 64 ? 32 : BS)
                            : P == SPAMM_BF16 ? (BS >= 128 ? 64 : BS)
                                              : (BS >= 128 ? 32 : BS);
  static constexpr int NSUB = LS / BS;    // tiles per side of a C leaf
  static constexpr int NPANEL = LS / KP;  // k-panels of one product
  static constexpr int NT = NW * 64;
  static constexpr int VN = 16 / ES;  // elements per 16-byte vector
  static constexpr int SA = KP + VN;  // padded row of an A (and BF16 B) panel in LDS
  static constexpr int KG = KP / NG;  // k values of one lane group per panel
  static constexpr int PV = BS * KP / VN;  // 16-byte vectors of one operand panel half
  static constexpr int A_VECS = (NH * PV + NT - 1) / NT;  // per thread (the last may be partial)
  static constexpr int B_VECS = A_VECS;
  static constexpr bool PARTIAL = (NH * PV) % NT != 0;
  static constexpr int A_LDS = NH * BS * SA * ES;               // bytes
  static constexpr int B_LDS = kBf ? NH * BS * SA * ES : KP * BS * ES;
  static constexpr int64_t LEAF_IN = int64_t(LS) * LS * (kBf ? 2 * ES : ES);  // bytes of a stored leaf
  static constexpr int64_t LEAF_OUT = int64_t(LS) * LS * sizeof(Out);
  static constexpr int VNO = 16 / int(sizeof(Out));
  static constexpr int SC = BS + VNO;  // padded row of the staged C leaf
  // double-buffered panels: a panel is stored into the buffer the panel
  // before last was read from, so one barrier per panel suffices
  static constexpr bool DBUF = (P == SPAMM_F32 && BS == 64 && LS == 64);
  static constexpr int PANEL_LDS = A_LDS + B_LDS;
  static constexpr int LDS = (DBUF ? 2 : 1) * PANEL_LDS;
  static constexpr bool STAGED = int64_t(BS) * SC * sizeof(Out) <= LDS;
  // FP32 accumulation in two levels: each leaf product is summed in its own
  // registers and then added to the leaf's total, so the rounding error of
  // a C entry grows with sqrt(bs) + sqrt(products) rather than with the
  // square root of all bs * products terms
  static constexpr bool TWO_LEVEL = P != SPAMM_F64;
  // resident workgroups per CU asked of the register allocator
  static constexpr int MINB = (BS == 64 && P == SPAMM_F32) ? 4 : (BS == 64 && P != SPAMM_F64) ? 3 : 1;
  static_assert(kBf ? KG % 8 == 0 : KG % 4 == 0, "lane group k slice");
  static_assert(LS % BS == 0 && LS % KP == 0 && NSUB <= 2, "tiles of a leaf");
};

template <int P, int MT>
struct AccSel {
  using type = f32x4;
};
template <>
struct AccSel<SPAMM_F64, 16> {
  using type = f64x4;
};
template <>
struct AccSel<SPAMM_F32, 32> {
  using type = f32x16;
};
template <>
struct AccSel<SPAMM_BF16, 32> {
  using type = f32x16;
};
template <>
struct AccSel<SPAMM_BF16X3, 32> {
  using type = f32x16;
};
template <int P, int BS, int V>
using Acc = typename AccSel<P, GemmCfg<P, BS, V>::MT>::type;
template <int P, int BS, int V>
using AccTiles = Acc<P, BS, V>[GemmCfg<P, BS, V>::TM][GemmCfg<P, BS, V>::TN];

// Row within an MFMA tile of accumulator register v held by lane group g:
// FP64 16x16x4: 4v + g (interleaved); FP32/BF16 16-wide: 4g + v;
// FP32/BF16 32-wide: 8(v/4) + 4g + v%4.
template <int P, int BS, int V>
__device__ __forceinline__ int acc_row(int g, int v) {
  if constexpr (GemmCfg<P, BS, V>::MT == 32) return 8 * (v / 4) + 4 * g + (v % 4);
  else if constexpr (P == SPAMM_F64) return 4 * v + g;
  else return 4 * g + v;
}

// FP32/FP64 B panel column swizzle of lane group g.
template <int P, int BS, int V>
__device__ __forceinline__ int b_swizzle(int g) {
  return (g * GemmCfg<P, BS, V>::MT) % BS;
}

// ---------------------------------------------------------------- unit records

// Scalar copy of one unit.
struct UnitS {
  int64_t pp;
  int32_t cnt, cidx, req, cf;
};

// Unit records live in a two-block LDS ring, 64 records per block: block
// `blk` holds units [u, u + 64) of the range.  Records are copied 8 bytes per
// thread (a record is three 8-byte words).
typedef int32_t i32x2r __attribute__((ext_vector_type(2)));
// The units a workgroup visits: visit t is unit ubase + (t / chunk) * cstride
// + t % chunk (chunks of `chunk` consecutive units, `cstride` apart).
struct Visits {
  int64_t ubase, cstride, chunk, n;
  __device__ __forceinline__ int64_t unit(int64_t t) const { return ubase + (t / chunk) * cstride + t % chunk; }
};

__device__ __forceinline__ void stage_recs(i32x2r (*ring)[64 * 3], int blk, const WorkUnit* __restrict__ wu,
                                           int64_t t0, const Visits& vs, int tid, int nt) {
  for (int w = tid; w < 64 * 3; w += nt) {
    const int64_t t = t0 + w / 3;
    if (t < vs.n) ring[blk][w] = *as_global(reinterpret_cast<const i32x2r*>(wu + vs.unit(t)) + (w % 3));
  }
}

__device__ __forceinline__ UnitS unit_of(const i32x2r (*ring)[64 * 3], int blk0, int64_t rel) {
  const int b = (blk0 + (rel >= 64 ? 1 : 0)) & 1;
  const int r = int(rel & 63);
  const i32x2r v0 = ring[b][3 * r], v1 = ring[b][3 * r + 1], v2 = ring[b][3 * r + 2];
  UnitS u;
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(v0[0]));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(v0[1]));
  u.pp = int64_t((uint64_t(hi) << 32) | lo);
  u.cnt = __builtin_amdgcn_readfirstlane(v1[0]);
  u.cidx = __builtin_amdgcn_readfirstlane(v1[1]);
  u.req = __builtin_amdgcn_readfirstlane(v2[0]);
  u.cf = __builtin_amdgcn_readfirstlane(v2[1]);
  return u;
}

// Leaf indices of 64 consecutive products of one unit, one product per lane.
struct Win {
  int32_t a, b;
};

__device__ __forceinline__ Win load_win(const char* __restrict__ base, const UnitS& u, int w, bool valid) {
  Win x;
  x.a = x.b = 0;
  const int i = w * 64 + (threadIdx.x & 63);
  if (valid && i < u.cnt) {
    const i32x2 v = *as_global(reinterpret_cast<const i32x2*>(base) + (u.pp + i));
    x.a = v[0];
    x.b = v[1];
  }
  return x;
}

// ---------------------------------------------------------------- panels

template <int P, int BS, int V>
struct Panel {
  u32x4 a[GemmCfg<P, BS, V>::A_VECS];
  u32x4 b[GemmCfg<P, BS, V>::B_VECS];
};

// k-panel `sub` of product (leaf ia of A, leaf ib of B) into registers; the
// unit's tile of C starts at row r0, column c0 of the leaf (0 unless the
// leaf holds several tiles).
template <int P, int BS, int V, int LS>
__device__ __forceinline__ void load_panel(Panel<P, BS, V>& r, const char* __restrict__ base, int32_t ia, int32_t ib,
                                           int sub, int r0, int c0, int tid) {
  using Cf = GemmCfg<P, BS, V, LS>;
  // wave-uniform leaf base plus a 32-bit lane offset (global loads with a
  // scalar base address)
  const auto A = as_global(base + int64_t(ia) * Cf::LEAF_IN);
  const auto B = as_global(base + int64_t(ib) * Cf::LEAF_IN);
#pragma unroll
  for (int t = 0; t < Cf::A_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    if (Cf::PARTIAL && v >= Cf::NH * Cf::PV) break;
    const int h = v / Cf::PV, vv = v % Cf::PV;
    const int row = vv / (Cf::KP / Cf::VN), cv = vv % (Cf::KP / Cf::VN);
    const uint32_t e = uint32_t(h * LS * LS + (r0 + row) * LS + sub * Cf::KP + cv * Cf::VN);  // uniform base + lane offset
    r.a[t] = *reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(A + uint32_t(e * Cf::ES));
  }
#pragma unroll
  for (int t = 0; t < Cf::B_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    if (Cf::PARTIAL && v >= Cf::NH * Cf::PV) break;
    uint32_t e;
    if constexpr (Cf::kBf) {  // transposed copy: row = B column, k contiguous
      const int h = v / Cf::PV, vv = v % Cf::PV;
      const int row = vv / (Cf::KP / Cf::VN), cv = vv % (Cf::KP / Cf::VN);
      e = uint32_t(h * LS * LS + (c0 + row) * LS + sub * Cf::KP + cv * Cf::VN);
    } else {
      const int kr = v / (BS / Cf::VN), cv = v % (BS / Cf::VN);
      e = uint32_t((sub * Cf::KP + kr) * LS + c0 + cv * Cf::VN);
    }
    r.b[t] = *reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(B + uint32_t(e * Cf::ES));
  }
}

template <int P, int BS, int V>
__device__ __forceinline__ void store_panel(const Panel<P, BS, V>& r, char* As, char* Bs, int tid) {
  using Cf = GemmCfg<P, BS, V>;
#pragma unroll
  for (int t = 0; t < Cf::A_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    if (Cf::PARTIAL && v >= Cf::NH * Cf::PV) break;
    const int h = v / Cf::PV, vv = v % Cf::PV;
    const int row = vv / (Cf::KP / Cf::VN), cv = vv % (Cf::KP / Cf::VN);
    *reinterpret_cast<u32x4*>(As + ((h * BS + row) * Cf::SA + cv * Cf::VN) * Cf::ES) = r.a[t];
  }
#pragma unroll
  for (int t = 0; t < Cf::B_VECS; ++t) {
    const int v = tid + t * Cf::NT;
    if (Cf::PARTIAL && v >= Cf::NH * Cf::PV) break;
    if constexpr (Cf::kBf) {
      const int h = v / Cf::PV, vv = v % Cf::PV;
      const int row = vv / (Cf::KP / Cf::VN), cv = vv % (Cf::KP / Cf::VN);
      *reinterpret_cast<u32x4*>(Bs + ((h * BS + row) * Cf::SA + cv * Cf::VN) * Cf::ES) = r.b[t];
    } else {
      const int kr = v / (BS / Cf::VN), cv = v % (BS / Cf::VN);
      const int sw = b_swizzle<P, BS, V>(kr / Cf::KG);
      *reinterpret_cast<u32x4*>(Bs + (kr * BS + ((cv * Cf::VN) ^ sw)) * Cf::ES) = r.b[t];
    }
  }
}

// One k-panel into the accumulators.
template <int P, int BS, int V>
__device__ __forceinline__ void compute_panel(AccTiles<P, BS, V>& acc, const char* As, const char* Bs, int row0, int col0, int li, int g) {
  using Cf = GemmCfg<P, BS, V>;
  if constexpr (Cf::kBf) {
#pragma unroll
    for (int s = 0; s < Cf::KG / 8; ++s) {
      const int k0 = g * Cf::KG + 8 * s;
      bf16x8 ah[Cf::TM], bh[Cf::TN], al[Cf::TM], bl[Cf::TN];
#pragma unroll
      for (int a = 0; a < Cf::TM; ++a) {
        const int o = (row0 + a * Cf::MT + li) * Cf::SA + k0;
        ah[a] = *reinterpret_cast<const bf16x8*>(As + o * 2);
        if constexpr (Cf::NH == 2) al[a] = *reinterpret_cast<const bf16x8*>(As + (o + BS * Cf::SA) * 2);
      }
#pragma unroll
      for (int b = 0; b < Cf::TN; ++b) {
        const int o = (col0 + b * Cf::MT + li) * Cf::SA + k0;
        bh[b] = *reinterpret_cast<const bf16x8*>(Bs + o * 2);
        if constexpr (Cf::NH == 2) bl[b] = *reinterpret_cast<const bf16x8*>(Bs + (o + BS * Cf::SA) * 2);
      }
#pragma unroll
      for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
        for (int b = 0; b < Cf::TN; ++b) {
          if constexpr (Cf::MT == 32) {
            if constexpr (Cf::NH == 2) {
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            }
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
          } else {
            if constexpr (Cf::NH == 2) {
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            }
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
          }
        }
    }
    // Wait states after the last BF16 MFMA before any later instruction may
    // overwrite its operand registers: with the window registers reused
    // right after the MFMA (a v_mov into its A-operand VGPRs a few cycles
    // after issue), a leaf-32 build returned wrong products.
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 7\n\ts_nop 7");
    __builtin_amdgcn_sched_barrier(0);
  } else {
    using T = typename std::conditional<P == SPAMM_F64, double, float>::type;
    const T* At = reinterpret_cast<const T*>(As);
    const T* Bt = reinterpret_cast<const T*>(Bs);
    const int swz = b_swizzle<P, BS, V>(g);
#pragma unroll 2
    for (int ch = 0; ch < Cf::KG / 4; ++ch) {
      const int kk = g * Cf::KG + 4 * ch;
      T av[Cf::TM][4];
      T bv[Cf::TN][4];
#pragma unroll
      for (int a = 0; a < Cf::TM; ++a) {
        const T* src = At + (row0 + a * Cf::MT + li) * Cf::SA + kk;
        if constexpr (P == SPAMM_F32) {
          const f32x4 x = *reinterpret_cast<const f32x4*>(src);
          av[a][0] = x[0];
          av[a][1] = x[1];
          av[a][2] = x[2];
          av[a][3] = x[3];
        } else {
          const f64x2 x0 = *reinterpret_cast<const f64x2*>(src);
          const f64x2 x1 = *reinterpret_cast<const f64x2*>(src + 2);
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
        for (int qq = 0; qq < 4; ++qq) bv[b][qq] = Bt[(kk + qq) * BS + col];
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
#pragma unroll
        for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
          for (int b = 0; b < Cf::TN; ++b) {
            if constexpr (P == SPAMM_F64)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][qq], bv[b][qq], acc[a][b], 0, 0, 0);
            else if constexpr (Cf::MT == 32)
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a][qq], bv[b][qq], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][qq], bv[b][qq], acc[a][b], 0, 0, 0);
          }
    }
  }
}

// ---------------------------------------------------------------- epilogue

template <int P, int BS, int V, int LS>
__device__ __forceinline__ void epilogue(const GemmArgs& ga, int64_t u, const UnitS& U, AccTiles<P, BS, V>& acc,
                                         char* smem,
                                         double* red, int tid, int lane, int wave, int row0, int col0, int li,
                                         int g) {
  using Cf = GemmCfg<P, BS, V, LS>;
  using Out = typename Cf::Out;
  // the unit's tile of the C leaf (the whole leaf unless LS > BS)
  const int tile = unit_tile(U.cf), tr0 = (tile / Cf::NSUB) * BS, tc0 = (tile % Cf::NSUB) * BS;
  const auto Cl = as_global(reinterpret_cast<Out*>(const_cast<char*>(ga.base) + int64_t(U.cidx) * Cf::LEAF_OUT) +
                            tr0 * LS + tc0);
  const uint32_t cm = uint32_t(U.cf & kUnitMorton);
  const bool has_ep = (U.cf & kUnitEp) != 0;
  Out alpha = Out(1), beta = Out(0);
  const Out* Dl = nullptr;
  if (has_ep) {  // requests with an epilogue read their descriptor here only
    const ReqDev* R = ga.reqs + U.req;
    alpha = Out(R->alpha);
    beta = Out(R->beta);
    if (R->Dslot != nullptr) {
      const int32_t ds = R->Dslot[cm];
      if (ds >= 0) Dl = static_cast<const Out*>(R->Dstore) + int64_t(ds) * LS * LS + tr0 * LS + tc0;
    }
  }
  uint32_t ci, cj;
  demorton(cm, ci, cj);
  Out* Cs = reinterpret_cast<Out*>(smem);
  double nsq = 0.0, tr = 0.0;
  if constexpr (Cf::STAGED) __syncthreads();  // every wave is done reading the panel buffers
#pragma unroll
  for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
    for (int b = 0; b < Cf::TN; ++b)
#pragma unroll
      for (int v = 0; v < Cf::AE; ++v) {
        const int row = row0 + a * Cf::MT + acc_row<P, BS, V>(g, v);
        const int col = col0 + b * Cf::MT + li;
        Out val = Out(acc[a][b][v]);
        if (has_ep) {
          const Out prod = alpha * val;
          const Out dv = Dl ? beta * as_global(Dl)[row * LS + col] : Out(0);
          val = prod + dv;
        }
        if constexpr (Cf::STAGED) Cs[row * Cf::SC + col] = val;
        else Cl[row * LS + col] = val;
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
  if constexpr (Cf::STAGED) {
    constexpr int NV = BS * BS / Cf::VNO / Cf::NT;
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int v = tid + t * Cf::NT;
      const int row = v / (BS / Cf::VNO), cv = v % (BS / Cf::VNO);
      *reinterpret_cast<__attribute__((address_space(1))) u32x4*>(Cl + row * LS + cv * Cf::VNO) =
          *reinterpret_cast<const u32x4*>(Cs + row * Cf::SC + cv * Cf::VNO);
    }
  }
  if (tid == 0) {
    double s = 0.0, t = 0.0;
    for (int x = 0; x < Cf::NW; ++x) {
      s += red[x];
      t += red[Cf::NW + x];
    }
    as_global(ga.wn)[u] = s;
    if (ci == cj && tr0 == tc0) as_global(ga.wt)[u] = t;  // a tile on the leaf's diagonal
  }
  // with double-buffered panels the next store is not preceded by a barrier:
  // every wave must be done reading the staged leaf first
  if constexpr (Cf::DBUF && Cf::STAGED) __syncthreads();
}

// ---------------------------------------------------------------- kernel

template <int P, int BS, int V, int LS>
__global__ void __launch_bounds__((GemmCfg<P, BS, V, LS>::NT), (GemmCfg<P, BS, V, LS>::MINB)) k_gemm(const GemmArgs ga) {
  using Cf = GemmCfg<P, BS, V, LS>;
  __shared__ __attribute__((aligned(16))) char smem[Cf::LDS];
  // per-wave partial sums of the epilogue, two sets used alternately: thread 0
  // may still read one set while the next unit's waves fill the other
  __shared__ double red2[2][2 * Cf::NW];
  int qg = 0;  // panels stored so far (picks the buffer when double-buffered)

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / Cf::WN, wc = wave % Cf::WN;
  const int row0 = wr * Cf::TILE_M, col0 = wc * Cf::TILE_N;
  const int li = lane % Cf::MT, g = lane / Cf::MT;
  const char* const base = ga.base;

  // the units this workgroup visits (visit t = 0 .. u1 - 1)
  const int xcd = int(blockIdx.x % kXcds), j = int(blockIdx.x / kXcds);
  Visits vs;
  if (ga.interleave > 0) {  // the XCD's share, dealt round-robin in chunks over its workgroups
    const int64_t lo = ga.start[xcd * ga.kx], hi = ga.start[(xcd + 1) * ga.kx];
    const int64_t c = ga.interleave, N = hi - lo, nch = (N + c - 1) / c;
    const int64_t mine = j < nch ? (nch - j + ga.kx - 1) / ga.kx : 0;  // chunks j, j + kx, ...
    vs.ubase = lo + int64_t(j) * c;
    vs.cstride = int64_t(ga.kx) * c;
    vs.chunk = c;
    vs.n = mine * c;
    if (mine > 0 && j + (mine - 1) * ga.kx == nch - 1 && N % c) vs.n -= c - N % c;  // the last chunk is partial
  } else {  // a contiguous range of equal cost
    const int rank = xcd * ga.kx + j;
    vs.ubase = ga.start[rank];
    vs.cstride = 0;
    vs.chunk = int64_t(1) << 62;
    vs.n = ga.start[rank + 1] - vs.ubase;
  }
  const int64_t u0 = 0, u1 = vs.n;
  if (u1 <= 0) return;

  // unit records of visits [rb, rb + 128) in the LDS ring (block blk0 first)
  __shared__ i32x2r ring[2][64 * 3];
  int64_t rb = u0;
  int blk0 = 0;
  stage_recs(ring, 0, ga.wu, rb, vs, tid, Cf::NT);
  stage_recs(ring, 1, ga.wu, rb + 64, vs, tid, Cf::NT);
  __syncthreads();

  // pair windows: W0 holds the window of the product being multiplied, W1
  // and W2 the next two windows of the range (unit by unit, 64 products
  // each; a unit without products has one empty window); (pu, pw) is W2's
  int64_t cu = u0;
  UnitS U = unit_of(ring, blk0, 0);
  Win W0 = load_win(base, U, 0, true);
  int64_t pu = cu;
  int pw = 0;
  UnitS PU = U;
  auto next_pos = [&]() {
    if ((pw + 1) * 64 < PU.cnt) {
      ++pw;
    } else {
      ++pu;
      pw = 0;
      if (pu < u1) PU = unit_of(ring, blk0, pu - rb);
    }
  };
  next_pos();
  Win W1 = load_win(base, PU, pw, pu < u1);
  next_pos();
  Win W2 = load_win(base, PU, pw, pu < u1);

  Panel<P, BS, V> pr;
  Win Wn;  // the window after W2, fetched early
  Wn.a = Wn.b = 0;
  bool wn_ready = false;
  // the current unit's tile within its C leaf (row and column offsets)
  int ur0 = (unit_tile(U.cf) / Cf::NSUB) * BS, uc0 = (unit_tile(U.cf) % Cf::NSUB) * BS;
  if (U.cnt > 0)
    load_panel<P, BS, V, LS>(pr, base, __builtin_amdgcn_readlane(W0.a, 0),
                              __builtin_amdgcn_readlane(W0.b, 0), 0, ur0, uc0, tid);

  for (;;) {
    const bool has_next = cu + 1 < u1;
    int32_t next_cnt = 0;
    int nr0 = 0, nc0 = 0;
    if (has_next) {
      const UnitS NU = unit_of(ring, blk0, cu + 1 - rb);
      next_cnt = NU.cnt;
      nr0 = (unit_tile(NU.cf) / Cf::NSUB) * BS;
      nc0 = (unit_tile(NU.cf) % Cf::NSUB) * BS;
    }

    Acc<P, BS, V> acc[Cf::TM][Cf::TN];
    Acc<P, BS, V> part[Cf::TWO_LEVEL ? Cf::TM : 1][Cf::TWO_LEVEL ? Cf::TN : 1];
#pragma unroll
    for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
      for (int b = 0; b < Cf::TN; ++b) acc[a][b] = Acc<P, BS, V>{};
    if constexpr (Cf::TWO_LEVEL) {
#pragma unroll
      for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
        for (int b = 0; b < Cf::TN; ++b) part[a][b] = Acc<P, BS, V>{};
    }

    for (int p = 0; p < U.cnt; ++p) {
      for (int sub = 0; sub < Cf::NPANEL; ++sub) {
        char* const As = smem + (Cf::DBUF ? (qg & 1) * Cf::PANEL_LDS : 0);
        char* const Bs = As + Cf::A_LDS;
        ++qg;
        // wave priorities: the panel's MFMAs 2, its store and the prefetch
        // loads 1, everything else (the epilogue's C writes) 0, so that of
        // the four workgroups on a SIMD the one with MFMA work ready issues
        // first and the next panels are staged ahead of epilogue traffic
        __builtin_amdgcn_s_setprio(1);
        if constexpr (!Cf::DBUF) __syncthreads();  // every wave is done with the previous panel
        store_panel<P, BS, V>(pr, As, Bs, tid);
        __syncthreads();
        // the window after W2 is fetched before the loads of the first panel
        // of the next window (loads complete in order, so waiting for that
        // panel does not wait on a window fetched later)
        if (!wn_ready && sub + 1 == Cf::NPANEL && (p + 1 == U.cnt || ((p + 1) & 63) == 0)) {
          next_pos();
          Wn = load_win(base, PU, pw, pu < u1);
          wn_ready = true;
        }
        // next panel: same product, next product (this or the next window),
        // or the first product of the next unit (the next window)
        if (sub + 1 < Cf::NPANEL) {
          load_panel<P, BS, V, LS>(pr, base, __builtin_amdgcn_readlane(W0.a, p & 63),
                                    __builtin_amdgcn_readlane(W0.b, p & 63), sub + 1, ur0, uc0, tid);
        } else if (p + 1 < U.cnt) {
          const int l = (p + 1) & 63;
          const bool nw = l == 0;
          const int32_t ia = nw ? __builtin_amdgcn_readlane(W1.a, 0) : __builtin_amdgcn_readlane(W0.a, l);
          const int32_t ib = nw ? __builtin_amdgcn_readlane(W1.b, 0) : __builtin_amdgcn_readlane(W0.b, l);
          load_panel<P, BS, V, LS>(pr, base, ia, ib, 0, ur0, uc0, tid);
        } else if (next_cnt > 0) {
          load_panel<P, BS, V, LS>(pr, base, __builtin_amdgcn_readlane(W1.a, 0),
                                    __builtin_amdgcn_readlane(W1.b, 0), 0, nr0, nc0, tid);
        }
        __builtin_amdgcn_s_setprio(2);
        if constexpr (Cf::TWO_LEVEL) {
          compute_panel<P, BS, V>(part, As, Bs, row0, col0, li, g);
          if (sub + 1 == Cf::NPANEL) {  // the product's sum joins the leaf's total
#pragma unroll
            for (int a = 0; a < Cf::TM; ++a)
#pragma unroll
              for (int b = 0; b < Cf::TN; ++b) {
                acc[a][b] += part[a][b];
                part[a][b] = Acc<P, BS, V>{};
              }
          }
        } else {
          compute_panel<P, BS, V>(acc, As, Bs, row0, col0, li, g);
        }
        __builtin_amdgcn_s_setprio(0);
      }
      if (((p + 1) & 63) == 0 && p + 1 < U.cnt) {  // into the unit's next window
        W0 = W1;
        W1 = W2;
        W2 = Wn;
        wn_ready = false;
      }
    }

    epilogue<P, BS, V, LS>(ga, vs.unit(cu), U, acc, smem, red2[cu & 1], tid, lane, wave, row0, col0, li, g);
    if (!has_next) break;

    const int32_t prev_cnt = U.cnt;
    ++cu;
    if (cu - rb == 64) {
      // units below cu are done: their block takes units [rb + 128, rb + 192),
      // first read some 60 units (and as many barriers) later
      rb += 64;
      blk0 ^= 1;
      stage_recs(ring, blk0 ^ 1, ga.wu, rb + 64, vs, tid, Cf::NT);
    }
    U = unit_of(ring, blk0, cu - rb);
    ur0 = nr0;
    uc0 = nc0;
    W0 = W1;
    W1 = W2;
    if (!wn_ready) {  // a unit without products fetched nothing ahead
      next_pos();
      Wn = load_win(base, PU, pw, pu < u1);
    }
    W2 = Wn;
    wn_ready = false;
    // the first panel of a unit that follows a unit without products was
    // not prefetched
    if (prev_cnt == 0 && U.cnt > 0)
      load_panel<P, BS, V, LS>(pr, base, __builtin_amdgcn_readlane(W0.a, 0),
                                __builtin_amdgcn_readlane(W0.b, 0), 0, ur0, uc0, tid);
  }
}

// ---------------------------------------------------------------- quads

// A quad (four sibling 64-leaves of C, see k_quad.hip) runs on a 128 x 128
// tile: the A panel stacks the A leaves of the two row halves and the B
// panel puts the B leaves of the two column halves side by side, so each
// staged leaf serves both children of its row (column).  Each child (2 *
// row half + column half) has its own waves, each a 32-column tile of it:
// two waves of 64 rows (two waves per SIMD), or for FP64 four of 32 rows
// (four per SIMD, so one's MFMAs run while the others wait on their
// operand reads).  A merged step is one k: the waves of the
// children that keep it add the product to their C leaf, the others only
// take part in the barriers.  Each child sums its own products k
// ascending, in the same panels and MFMA order whatever its siblings keep.
//
// Panels move from memory to LDS by direct loads (global_load_lds, 16 bytes
// per lane, no registers) into a ring of four stages: two panels are
// multiplied per barrier while the next two load, so a group's loads wait
// on the memory latency while the group before it is multiplied.  A leaf
// no child of the step needs is replaced by its partner's in the plan, so
// every panel is the same loads and a wave's wait for a group is a count
// of its later loads.  FP64 issues a group at once (one read of the step);
// the eight-wave kernels issue panel by panel, which their compiled loops
// run faster.  A stage is 16 KiB of A and 16 KiB of B.  A row of the A
// part (and of transposed BF16 B) is the panel's k of one row, its 16-byte
// chunks XOR-swizzled by row so that the operand reads of consecutive rows
// fall on different banks; FP32 / FP64 B is k-major, one 64-column block
// per B leaf, its columns swizzled by lane group.  Each load instruction
// reads one leaf: a scalar leaf address plus a fixed per-lane offset.

template <int P, int V, int RS = 64>
struct QuadCfg {
  using G = GemmCfg<P, 128, V>;
  static constexpr bool kBf = G::kBf;
  static constexpr int NH = G::NH, ES = G::ES, MT = G::MT, NG = G::NG, AE = G::AE;
  static constexpr bool TWO_LEVEL = G::TWO_LEVEL;
  // waves: FP64 four per child (32 x 32 of it each, four waves per SIMD to
  // hide the operand reads: 2% faster than two), the others two (64 x 32)
  static constexpr int NW = P == SPAMM_F64 ? 16 : 8, NT = NW * 64;
  static constexpr int WPC = NW / 4;                 // waves per child
  static constexpr int TILE_M = WPC == 4 ? 32 : 64, TILE_N = 32;  // a wave's part of its child
  static constexpr int TM = TILE_M / MT, TN = TILE_N / MT;
  static constexpr int PART = 16384;                 // bytes of the A (or B) part of a stage
  static constexpr int KP = PART / (128 * ES * NH);  // k per panel: 64 BF16, 32 BF16X3 / FP32, 16 FP64
  static constexpr int NP = 64 / KP;                 // panels per 64-leaf product
  static constexpr int KG = KP / NG;                 // k of one lane group per panel
  static constexpr int RB = KP * ES;                 // bytes of an A row (or a transposed B row)
  static constexpr int CH = RB / 16;                 // 16-byte chunks per row
  static constexpr int VN = 16 / ES;                 // elements per chunk
  static constexpr int STAGE = 2 * PART;
  static constexpr int NSTAGE = 4;
  // panels multiplied between two barriers, the next GP loading meanwhile
  // (BF16, one panel per product, has its quads' step counts padded to even)
  static constexpr int GP = 2;
  static constexpr int VPT = PART / 1024 / NW;       // 1 KiB load blocks of a part per wave
  static constexpr int LOADS = 2 * VPT;              // load instructions per wave per panel
  // stored leaves of side RS: 64 (the quad's children are four C leaves),
  // or 128 / 256 (the quad is a 128 x 128 tile of one C leaf, its children
  // the tile's four 64 x 64 blocks)
  static constexpr int64_t LEAF = int64_t(RS) * RS * (kBf ? 2 * ES : ES);  // bytes of a stored leaf
  // the unit of a step's operand indices: whole leaves at RS = 64, else
  // 64-element offsets from the arena base (the start of a 64 x 64 block)
  static constexpr int64_t UNIT = RS == 64 ? LEAF : int64_t(64) * ES;
  static constexpr int NSUB = RS / 128;  // 128-tiles per side of a C leaf (RS > 64)
  static_assert(CH >= 1 && CH <= 8 && 8 % CH == 0, "row chunks");
  static_assert(kBf ? KG % 8 == 0 : KG % 4 == 0, "lane group k slice");
  static_assert(VPT * NW * 1024 == PART, "whole load blocks per part");
  static_assert(MT == 16, "quads take 16 x 16 MFMA tiles");
  static_assert(RS == 64 || RS == 128 || RS == 256, "leaf sides of the quad kernel");
  static_assert((NP % GP == 0 || NP == 1) && NSTAGE == 2 * GP, "panel groups: one step, or GP steps; two groups in the ring");
};

template <int P, int V>
using QAcc = Acc<P, 128, V>[QuadCfg<P, V>::TM][QuadCfg<P, V>::TN];

// Physical chunk of logical chunk kc in row R of an A (or transposed B)
// part: 8 consecutive rows take 8 different 16-byte bank groups.
template <int CH>
__device__ __forceinline__ int qswz(int R) {
  return (R / (8 / CH)) % CH;
}

// Scalar copy of one quad record (global memory, the range's quad q).
struct QuadS {
  int64_t sp;
  int32_t ns, u0, cmask, req;
};

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  return int64_t((uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int32_t(uint64_t(v) >> 32)))) << 32) |
                 uint32_t(__builtin_amdgcn_readfirstlane(int32_t(uint64_t(v) & 0xffffffffu))));
}

__device__ __forceinline__ QuadS quad_at(const GemmArgs& ga, int64_t q) {
  const QuadUnit* p = ga.qu + q;
  QuadS r;
  r.sp = uniform64(p->sp);
  r.ns = __builtin_amdgcn_readfirstlane(p->ns);
  r.u0 = __builtin_amdgcn_readfirstlane(p->u0);
  r.cmask = __builtin_amdgcn_readfirstlane(p->cmask);
  r.req = __builtin_amdgcn_readfirstlane(p->req);
  return r;
}

// Operand leaves and children of 64 consecutive steps, one step per lane.
struct Win4 {
  int32_t a0, a1, b0, b1, m;
};

__device__ __forceinline__ Win4 load_win4(const GemmArgs& ga, int64_t sp, int32_t ns, int w, bool valid) {
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  Win4 x;
  x.a0 = x.a1 = x.b0 = x.b1 = -1;
  x.m = 0;
  const int i = w * 64 + (threadIdx.x & 63);
  if (valid && i < ns) {
    const i32x4 v = *as_global(reinterpret_cast<const i32x4*>(ga.steps) + (sp + i));
    x.a0 = v[0];
    x.a1 = v[1];
    x.b0 = v[2];
    x.b1 = v[3];
    x.m = int32_t(*as_global(ga.smask + (sp + i)));
  }
  return x;
}

// Per-lane byte offsets (within a leaf, panel 0) of the wave's load blocks.
template <int P, int V, int RS>
struct QuadOffs {
  uint32_t a[QuadCfg<P, V, RS>::VPT], b[QuadCfg<P, V, RS>::VPT];
};

template <int P, int V, int RS>
__device__ __forceinline__ QuadOffs<P, V, RS> quad_offsets(int wave, int lane) {
  using Q = QuadCfg<P, V, RS>;
  QuadOffs<P, V, RS> o;
#pragma unroll
  for (int i = 0; i < Q::VPT; ++i) {
    const int q = (i * Q::NW + wave) * 64 + lane;  // chunk of the part
    {
      const int R = q / Q::CH, phys = q % Q::CH;
      const int h = R / 128, r = R % 128;
      const int kc = phys ^ qswz<Q::CH>(R);
      o.a[i] = uint32_t((h * RS * RS + (r & 63) * RS + kc * Q::VN) * Q::ES);
    }
    if constexpr (Q::kBf) {  // transposed copy: a row is a B column, k contiguous
      const int R = q / Q::CH, phys = q % Q::CH;
      const int h = R / 128, r = R % 128;
      const int kc = phys ^ qswz<Q::CH>(R);
      o.b[i] = uint32_t((h * RS * RS + (r & 63) * RS + kc * Q::VN) * Q::ES);
    } else {  // k-major: one 64-column block per leaf, row kr of 64 columns
      const int qh = q % (Q::KP * 64 / Q::VN);
      const int kr = qh / (64 / Q::VN), pc = (qh % (64 / Q::VN)) * Q::VN;
      const int col = pc ^ (((kr / Q::KG) * Q::MT) % 64);
      o.b[i] = uint32_t((kr * RS + col) * Q::ES);
    }
  }
  return o;
}

// Direct loads of k-panel `sub` of a step (leaves a0 / a1 of the A row
// halves, b0 / b1 of the B column halves; the plan has put a partner's leaf
// where no child of the step needs one) into stage `st`.
template <int P, int V, int RS>
__device__ __forceinline__ void issue_panel(char* st, const char* __restrict__ base, const QuadOffs<P, V, RS>& o,
                                            int32_t a0, int32_t a1, int32_t b0, int32_t b1, int sub, int wave) {
  using Q = QuadCfg<P, V, RS>;
  // FP64 (and every precision on large leaves, whose block offsets may
  // exceed 2^31) takes the plan's indices as they are, unsigned (the fewest
  // scalar instructions); the eight-wave kernels on 64-leaves keep the
  // signed form with the partner check, a no-op after the plan but
  // measured to schedule better there
  constexpr bool kLean = P == SPAMM_F64 || RS > 64;
  using LT = std::conditional_t<kLean, uint32_t, int32_t>;
  using OT = std::conditional_t<kLean, uint64_t, int64_t>;
  using ST = std::conditional_t<kLean, uint32_t, int64_t>;
  if constexpr (!kLean) {
    if (a0 < 0) a0 = a1;
    if (a1 < 0) a1 = a0;
    if (b0 < 0) b0 = b1;
    if (b1 < 0) b1 = b0;
  }
#pragma unroll
  for (int i = 0; i < Q::VPT; ++i) {
    const int blk = i * Q::NW + wave;  // 1 KiB block of the part (wave-uniform)
    // an A block's rows lie in one row half
    const LT leaf = ((blk * 64 / Q::CH) % 128) < 64 ? a0 : a1;
    const auto L = as_global(base + OT(leaf) * Q::UNIT + sub * (Q::KP * Q::ES));
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const __attribute__((address_space(1))) void*>(L + o.a[i]),
                                     (__attribute__((address_space(3))) void*)(st + blk * 1024), 16, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < Q::VPT; ++i) {
    const int blk = i * Q::NW + wave;
    LT leaf;
    ST so;
    if constexpr (Q::kBf) {
      leaf = ((blk * 64 / Q::CH) % 128) < 64 ? b0 : b1;
      so = sub * (Q::KP * Q::ES);
    } else {
      leaf = blk < 8 ? b0 : b1;  // blocks 0-7: the left B leaf, 8-15: the right
      so = ST(sub) * ST(Q::KP * RS * Q::ES);
    }
    const auto L = as_global(base + OT(leaf) * Q::UNIT + so);
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const __attribute__((address_space(1))) void*>(L + o.b[i]),
                                     (__attribute__((address_space(3))) void*)(st + Q::PART + blk * 1024), 16, 0, 0);
  }
}

// Wait until at most n of this wave's loads are outstanding (the loads of
// the panels issued after the ones wanted).
__device__ __forceinline__ void wait_loads(int n) {
  switch (n) {
    case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
    case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    case 6: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
    case 8: asm volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
    default: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
  }
}

// Workgroup barrier that orders LDS accesses at the compiler level only
// (the direct loads it waits for were counted explicitly).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// One k-panel of the stage at As / Bs into the accumulators of the wave's
// tile (rows row0.., columns col0.. of the 128 x 128 quad).
template <int P, int V>
__device__ __forceinline__ void compute_quad_panel(QAcc<P, V>& acc, const char* As, const char* Bs, int row0,
                                                   int col0, int li, int g) {
  using Q = QuadCfg<P, V>;
  if constexpr (Q::kBf) {
#pragma unroll
    for (int s = 0; s < Q::KG / 8; ++s) {
      const int kc = (g * Q::KG + 8 * s) / 8;
      bf16x8 ah[Q::TM], bh[Q::TN], al[Q::TM], bl[Q::TN];
#pragma unroll
      for (int a = 0; a < Q::TM; ++a) {
        const int R = row0 + a * Q::MT + li;
        const int o = R * Q::RB + ((kc ^ qswz<Q::CH>(R)) << 4);
        ah[a] = *reinterpret_cast<const bf16x8*>(As + o);
        if constexpr (Q::NH == 2) al[a] = *reinterpret_cast<const bf16x8*>(As + 128 * Q::RB + o);
      }
#pragma unroll
      for (int b = 0; b < Q::TN; ++b) {
        const int R = col0 + b * Q::MT + li;
        const int o = R * Q::RB + ((kc ^ qswz<Q::CH>(R)) << 4);
        bh[b] = *reinterpret_cast<const bf16x8*>(Bs + o);
        if constexpr (Q::NH == 2) bl[b] = *reinterpret_cast<const bf16x8*>(Bs + 128 * Q::RB + o);
      }
#pragma unroll
      for (int a = 0; a < Q::TM; ++a)
#pragma unroll
        for (int b = 0; b < Q::TN; ++b) {
          if constexpr (Q::NH == 2) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          }
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
    // the BF16 operand-read wait states (as in compute_panel)
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 7\n\ts_nop 7");
    __builtin_amdgcn_sched_barrier(0);
  } else {
    using T = typename std::conditional<P == SPAMM_F64, double, float>::type;
    const T* Bt = reinterpret_cast<const T*>(Bs);
    const int swz = (g * Q::MT) % 64;
#pragma unroll 2
    for (int ch = 0; ch < Q::KG / 4; ++ch) {
      const int kk = g * Q::KG + 4 * ch;
      T av[Q::TM][4];
      T bv[Q::TN][4];
#pragma unroll
      for (int a = 0; a < Q::TM; ++a) {
        const int R = row0 + a * Q::MT + li;
        if constexpr (P == SPAMM_F32) {
          const int o = R * Q::RB + (((kk / 4) ^ qswz<Q::CH>(R)) << 4);
          const f32x4 x = *reinterpret_cast<const f32x4*>(As + o);
          av[a][0] = x[0];
          av[a][1] = x[1];
          av[a][2] = x[2];
          av[a][3] = x[3];
        } else {
          const int o0 = R * Q::RB + (((kk / 2) ^ qswz<Q::CH>(R)) << 4);
          const int o1 = R * Q::RB + (((kk / 2 + 1) ^ qswz<Q::CH>(R)) << 4);
          const f64x2 x0 = *reinterpret_cast<const f64x2*>(As + o0);
          const f64x2 x1 = *reinterpret_cast<const f64x2*>(As + o1);
          av[a][0] = x0[0];
          av[a][1] = x0[1];
          av[a][2] = x1[0];
          av[a][3] = x1[1];
        }
      }
#pragma unroll
      for (int b = 0; b < Q::TN; ++b) {
        const int c = col0 + b * Q::MT + li;  // column of the quad
        const T* blk = Bt + (c >> 6) * (Q::KP * 64);
        const int cc = (c & 63) ^ swz;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) bv[b][qq] = blk[(kk + qq) * 64 + cc];
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
#pragma unroll
        for (int a = 0; a < Q::TM; ++a)
#pragma unroll
          for (int b = 0; b < Q::TN; ++b) {
            if constexpr (P == SPAMM_F64)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][qq], bv[b][qq], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][qq], bv[b][qq], acc[a][b], 0, 0, 0);
          }
    }
  }
}

// The C blocks of a quad from the waves' accumulators: C (optionally
// alpha * AB + beta * D), its FP64 squared norm and, on the diagonal, its
// diagonal sum, for the work unit (a child's C leaf at RS = 64, else the
// quad's 128 x 128 tile of one C leaf).  Called by every wave at the same
// point (it holds a workgroup barrier); red: 2 * NW partial sums.
template <int P, int V, int RS>
__device__ __forceinline__ void epilogue_quad(const GemmArgs& ga, const QuadS& q, QAcc<P, V>& acc, double* red,
                                              int wave, int lane, int child, int crow0, int ccol0, int li,
                                              int g) {
  using Q = QuadCfg<P, V, RS>;
  using Out = typename GemmCfg<P, 128, V>::Out;
  const bool present = RS > 64 || ((q.cmask >> child) & 1);
  const int64_t u =
      RS > 64 ? int64_t(q.u0) : int64_t(q.u0) + __builtin_popcount(uint32_t(q.cmask) & ((1u << child) - 1u));
  uint32_t ci = 0, cj = 0;
  int r0 = 0, c0 = 0;  // the child's block in its C leaf
  bool diag_tile = true;
  if (present) {
    const WorkUnit W = ga.wu[u];
    const auto Cl =
        as_global(reinterpret_cast<Out*>(const_cast<char*>(ga.base) + int64_t(W.cidx) * RS * RS * sizeof(Out)));
    const uint32_t cm = uint32_t(W.cflags & kUnitMorton);
    if constexpr (RS > 64) {
      const int tile = unit_tile(W.cflags);
      const int tr0 = (tile / Q::NSUB) * 128, tc0 = (tile % Q::NSUB) * 128;
      diag_tile = tr0 == tc0;
      r0 = tr0 + 64 * (child >> 1);
      c0 = tc0 + 64 * (child & 1);
    }
    const bool has_ep = (W.cflags & kUnitEp) != 0;
    Out alpha = Out(1), beta = Out(0);
    const Out* Dl = nullptr;
    if (has_ep) {
      const ReqDev* R = ga.reqs + W.req;
      alpha = Out(R->alpha);
      beta = Out(R->beta);
      if (R->Dslot != nullptr) {
        const int32_t ds = R->Dslot[cm];
        if (ds >= 0) Dl = static_cast<const Out*>(R->Dstore) + int64_t(ds) * RS * RS;
      }
    }
    demorton(cm, ci, cj);
    double nsq = 0.0, tr = 0.0;
#pragma unroll
    for (int a = 0; a < Q::TM; ++a)
#pragma unroll
      for (int b = 0; b < Q::TN; ++b)
#pragma unroll
        for (int v = 0; v < Q::AE; ++v) {
          const int row = r0 + crow0 + a * Q::MT + acc_row<P, 128, V>(g, v);  // within the C leaf
          const int col = c0 + ccol0 + b * Q::MT + li;
          Out val = Out(acc[a][b][v]);
          if (has_ep) {
            const Out prod = alpha * val;
            const Out dv = Dl ? beta * as_global(Dl)[row * RS + col] : Out(0);
            val = prod + dv;
          }
          Cl[row * RS + col] = val;
          const double dval = double(val);
          nsq += dval * dval;
          if (row == col) tr += dval;
        }
    nsq = wave_sum_f64(nsq);
    tr = wave_sum_f64(tr);
    if (lane == 0) {
      red[wave] = nsq;
      red[Q::NW + wave] = tr;
    }
  }
  __syncthreads();
  // the unit's parts, in wave order: a child's waves at RS = 64, every wave
  // of the quad else
  constexpr int WPU = RS > 64 ? Q::NW : Q::WPC;
  if (present && wave % WPU == 0 && lane == 0) {
    double s = 0.0, t = 0.0;
#pragma unroll
    for (int x = 0; x < WPU; ++x) {
      s += red[wave + x];
      t += red[Q::NW + wave + x];
    }
    as_global(ga.wn)[u] = s;
    if (ci == cj && diag_tile) as_global(ga.wt)[u] = t;
  }
}

template <int P, int V, int RS>
__global__ void __launch_bounds__((QuadCfg<P, V, RS>::NT), 1) k_gemm_quad(const GemmArgs ga) {
  using Q = QuadCfg<P, V, RS>;
  __shared__ __attribute__((aligned(1024))) char smem[Q::NSTAGE * Q::STAGE];
  // partial norm and diagonal sums of the epilogue, two sets used in turn
  __shared__ double red2[2][2 * Q::NW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int child = wave / Q::WPC;  // the C leaf (2 * row half + column half) this wave works on
  const int part_ = wave % Q::WPC;
  const int crow0 = (part_ / 2) * Q::TILE_M, ccol0 = (part_ % 2) * Q::TILE_N;  // the wave's tile in the child
  const int row0 = (child >> 1) * 64 + crow0, col0 = (child & 1) * 64 + ccol0;  // ... and in the quad
  const int li = lane % Q::MT, g = lane / Q::MT;
  const char* const base = ga.base;
  const QuadOffs<P, V, RS> offs = quad_offsets<P, V, RS>(wave, lane);

  // the quads this workgroup visits (visit t = 0 .. u1 - 1): a contiguous
  // range of equal cost, or the XCD's share dealt round-robin over its
  // workgroups in chunks (Morton-adjacent quads running together share
  // their operand leaves in the XCD's L2); ranges are cut at the number of
  // quads, known on the device only
  const int xcd = int(blockIdx.x % kXcds), j = int(blockIdx.x / kXcds);
  const int64_t nq = *ga.nq;
  Visits vs;
  if (ga.interleave > 0) {
    const int64_t lo = min(ga.start[xcd * ga.kx], nq), hi = min(ga.start[(xcd + 1) * ga.kx], nq);
    const int64_t c = ga.interleave, N = hi - lo, nch = (N + c - 1) / c;
    const int64_t mine = j < nch ? (nch - j + ga.kx - 1) / ga.kx : 0;  // chunks j, j + kx, ...
    vs.ubase = lo + int64_t(j) * c;
    vs.cstride = int64_t(ga.kx) * c;
    vs.chunk = c;
    vs.n = mine * c;
    if (mine > 0 && j + (mine - 1) * ga.kx == nch - 1 && N % c) vs.n -= c - N % c;  // the last chunk is partial
  } else {
    const int rank = xcd * ga.kx + j;
    vs.ubase = ga.start[rank];
    vs.cstride = 0;
    vs.chunk = int64_t(1) << 62;
    vs.n = min(ga.start[rank + 1], nq) - vs.ubase;
  }
  const int64_t u1 = vs.n;
  if (u1 <= 0) return;
  const GemmArgs* gp = &ga;
  auto rec = [&](int64_t t) {
    if constexpr (P == SPAMM_F64)  // (contiguous ranges need no division)
      return quad_at(*gp, vs.cstride == 0 ? vs.ubase + t : vs.unit(t));
    else
      return quad_at(*gp, vs.unit(t));
  };

  // loader: quad lq (with steps), step ls, panel lsub; WL holds the window of
  // step ls, WN the window after it, at (pq, pw)
  int64_t lq = 0;
  QuadS LQ = rec(0);
  while (LQ.ns == 0 && ++lq < u1) LQ = rec(lq);
  bool lmore = lq < u1;
  int32_t ls = 0;
  int lsub = 0;
  Win4 WL = load_win4(ga, LQ.sp, LQ.ns, 0, lmore);
  int64_t pq = lq;
  int pw = 0;
  QuadS PQ = LQ;
  auto next_win = [&]() {  // (pq, pw) to the next window of a quad with steps
    if ((pw + 1) * 64 < PQ.ns) {
      ++pw;
    } else {
      pw = 0;
      do {
        ++pq;
        if (pq < u1) PQ = rec(pq);
      } while (pq < u1 && PQ.ns == 0);
    }
    pq = uniform64(pq);
    pw = __builtin_amdgcn_readfirstlane(pw);
  };
  if (lmore) next_win();
  Win4 WN = load_win4(ga, PQ.sp, PQ.ns, pw, lmore && pq < u1);

  // per panel in flight (up to four, one byte each, oldest lowest): the
  // children that keep its step
  uint32_t fifo = 0;
  int ahead = 0, ist = 0, cst = 0;  // panels in flight, next stage to fill, stage to multiply
  auto next_step = [&](int by) {     // ls += by (the steps stay in one window and one quad)
    ls += by;
    if (ls == LQ.ns) {  // the next quad with steps: its first window is WN
      lq = pq;
      LQ = PQ;
      ls = 0;
      lmore = lq < u1;
      WL = WN;
      if (lmore) {
        next_win();
        WN = load_win4(*gp, PQ.sp, PQ.ns, pw, pq < u1);
      }
    } else if ((ls & 63) == 0) {  // the quad's next window
      WL = WN;
      next_win();
      WN = load_win4(*gp, PQ.sp, PQ.ns, pw, pq < u1);
    }
  };
  // the next panel of the stream into stage ist
  auto issue_one = [&]() {
    const int l = ls & 63;
    const int32_t a0 = __builtin_amdgcn_readlane(WL.a0, l), a1 = __builtin_amdgcn_readlane(WL.a1, l);
    const int32_t b0 = __builtin_amdgcn_readlane(WL.b0, l), b1 = __builtin_amdgcn_readlane(WL.b1, l);
    const uint32_t m = uint32_t(__builtin_amdgcn_readlane(WL.m, l));
    issue_panel<P, V, RS>(smem + ist * Q::STAGE, base, offs, a0, a1, b0, b1, lsub, wave);
    const bool last_sub = lsub + 1 == Q::NP;
    fifo |= m << (8 * ahead);
    ++ahead;
    ist = (ist + 1) % Q::NSTAGE;
    if (!last_sub) {
      ++lsub;
    } else {
      lsub = 0;
      ++ls;
      if (ls == LQ.ns) {  // the next quad with steps: its first window is WN
        lq = pq;
        LQ = PQ;
        ls = 0;
        lmore = lq < u1;
        WL = WN;
        if (lmore) {
          next_win();
          WN = load_win4(*gp, PQ.sp, PQ.ns, pw, pq < u1);
        }
      } else if ((ls & 63) == 0) {  // the quad's next window
        WL = WN;
        next_win();
        WN = load_win4(*gp, PQ.sp, PQ.ns, pw, pq < u1);
      }
    }
  };
  // the next GP panels of the stream into stages ist, ist + 1: GP k-panels
  // of one step, or (one panel per product) GP steps, which share a window
  // (the step counts are even)
  auto issue_group = [&]() {
    char* const st = smem + ist * Q::STAGE;
    if constexpr (Q::NP % Q::GP == 0) {
      const int l = ls & 63;
      const int32_t a0 = __builtin_amdgcn_readlane(WL.a0, l), a1 = __builtin_amdgcn_readlane(WL.a1, l);
      const int32_t b0 = __builtin_amdgcn_readlane(WL.b0, l), b1 = __builtin_amdgcn_readlane(WL.b1, l);
      const uint32_t m = uint32_t(__builtin_amdgcn_readlane(WL.m, l));
#pragma unroll
      for (int k = 0; k < Q::GP; ++k) {
        issue_panel<P, V, RS>(st + k * Q::STAGE, base, offs, a0, a1, b0, b1, lsub + k, wave);
        fifo |= m << (8 * (ahead + k));
      }
      lsub += Q::GP;
      if (lsub == Q::NP) {
        lsub = 0;
        next_step(1);
      }
    } else {
#pragma unroll
      for (int k = 0; k < Q::GP; ++k) {
        const int l = (ls + k) & 63;
        const int32_t a0 = __builtin_amdgcn_readlane(WL.a0, l), a1 = __builtin_amdgcn_readlane(WL.a1, l);
        const int32_t b0 = __builtin_amdgcn_readlane(WL.b0, l), b1 = __builtin_amdgcn_readlane(WL.b1, l);
        const uint32_t m = uint32_t(__builtin_amdgcn_readlane(WL.m, l));
        issue_panel<P, V, RS>(st + k * Q::STAGE, base, offs, a0, a1, b0, b1, 0, wave);
        fifo |= m << (8 * (ahead + k));
      }
      next_step(Q::GP);
    }
    ahead += Q::GP;
    ist = (ist + Q::GP) & (Q::NSTAGE - 1);
  };

  QAcc<P, V> acc;
  auto clear = [&]() {
#pragma unroll
    for (int a = 0; a < Q::TM; ++a)
#pragma unroll
      for (int b = 0; b < Q::TN; ++b) acc[a][b] = Acc<P, 128, V>{};
  };
  clear();

  // quads without steps (C from the epilogue alone, zero products) up to the
  // next quad with steps
  int64_t cq = 0;
  auto flush_empty = [&]() {
    while (cq < u1) {
      const QuadS E = rec(cq);
      if (E.ns != 0) break;
      epilogue_quad<P, V, RS>(*gp, E, acc, red2[cq & 1], wave, lane, child, crow0, ccol0, li, g);
      ++cq;
    }
  };
  flush_empty();

  // the loader: FP64 (sixteen waves) reads a group's steps once, the
  // eight-wave kernels panel by panel (each measured faster that way)
  auto issue_next = [&]() {
    if constexpr (P == SPAMM_F64) {
      if (lmore) issue_group();
    } else {
#pragma unroll
      for (int k = 0; k < Q::GP; ++k)
        if (lmore) issue_one();
    }
  };
  if constexpr (P == SPAMM_F64) {
    if (lmore) issue_group();
  } else {
    for (int i = 0; i < Q::NSTAGE - Q::GP && lmore; ++i) issue_one();
  }
  // the quads with steps in order, each over its panels (the loader issued
  // exactly these panels in this order), GP panels per barrier
  while (cq < u1) {
    const QuadS C = rec(cq);
    const int32_t npan = C.ns * Q::NP;
    for (int32_t p = 0; p < npan; p += Q::GP) {
      // loop state is wave-uniform: keep it in scalar registers
      ahead = __builtin_amdgcn_readfirstlane(ahead);
      fifo = uint32_t(__builtin_amdgcn_readfirstlane(int32_t(fifo)));
      ist = __builtin_amdgcn_readfirstlane(ist);
      cst = __builtin_amdgcn_readfirstlane(cst);
      ls = __builtin_amdgcn_readfirstlane(ls);
      lsub = __builtin_amdgcn_readfirstlane(lsub);
      lmore = __builtin_amdgcn_readfirstlane(int32_t(lmore)) != 0;
      // this wave's loads of the oldest GP panels are in LDS (FP64: all it
      // issued, the ring holding two groups)
      if constexpr (P == SPAMM_F64)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      else
        wait_loads((ahead - Q::GP) * Q::LOADS);
      lds_barrier();  // every wave's are, and the stages multiplied last are free
      uint32_t meta[Q::GP];
      int st[Q::GP];
#pragma unroll
      for (int k = 0; k < Q::GP; ++k) {  // the oldest panels leave the queue
        meta[k] = fifo & 0xffu;
        fifo >>= 8;
        if constexpr (P == SPAMM_F64) {
          st[k] = cst + k;  // (a group's stages are adjacent)
        } else {
          st[k] = cst;
          cst = (cst + 1) % Q::NSTAGE;
        }
      }
      if constexpr (P == SPAMM_F64) cst = (cst + Q::GP) & (Q::NSTAGE - 1);
      ahead -= Q::GP;
      issue_next();  // the next group, into the stages multiplied last
      // a wave whose child does not keep a step skips it (its SIMD partner,
      // another child's wave, has the matrix core to itself)
      if constexpr (!Q::TWO_LEVEL) {  // FP64: one level; the group is two panels of one step
        static_assert(Q::NP % Q::GP == 0, "a group within one step");
        if ((meta[0] >> child) & 1u) {
#pragma unroll
          for (int k = 0; k < Q::GP; ++k)
            compute_quad_panel<P, V>(acc, smem + st[k] * Q::STAGE, smem + st[k] * Q::STAGE + Q::PART, row0, col0,
                                     li, g);
        }
      } else if constexpr (Q::NP == 1) {  // BF16: a product per panel, its sum from zero
#pragma unroll
        for (int k = 0; k < Q::GP; ++k)
          if ((meta[k] >> child) & 1u) {
            QAcc<P, V> part;
#pragma unroll
            for (int a = 0; a < Q::TM; ++a)
#pragma unroll
              for (int b = 0; b < Q::TN; ++b) part[a][b] = Acc<P, 128, V>{};
            compute_quad_panel<P, V>(part, smem + st[k] * Q::STAGE, smem + st[k] * Q::STAGE + Q::PART, row0,
                                     col0, li, g);
#pragma unroll
            for (int a = 0; a < Q::TM; ++a)
#pragma unroll
              for (int b = 0; b < Q::TN; ++b) acc[a][b] += part[a][b];
          }
      } else {  // the group is one product (both panels of one step)
        if ((meta[0] >> child) & 1u) {
          QAcc<P, V> part;
#pragma unroll
          for (int a = 0; a < Q::TM; ++a)
#pragma unroll
            for (int b = 0; b < Q::TN; ++b) part[a][b] = Acc<P, 128, V>{};
#pragma unroll
          for (int k = 0; k < Q::GP; ++k)
            compute_quad_panel<P, V>(part, smem + st[k] * Q::STAGE, smem + st[k] * Q::STAGE + Q::PART, row0,
                                     col0, li, g);
#pragma unroll
          for (int a = 0; a < Q::TM; ++a)
#pragma unroll
            for (int b = 0; b < Q::TN; ++b) acc[a][b] += part[a][b];
        }
      }
    }
    epilogue_quad<P, V, RS>(ga, C, acc, red2[cq & 1], wave, lane, child, crow0, ccol0, li, g);
    clear();
    ++cq;
    flush_empty();
  }
}

template <int P, int V>
static int max_groups_quad(int n_cu) {
  static const int per_cu = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_gemm_quad<P, V, 64>, QuadCfg<P, V>::NT, 0) != hipSuccess ||
        v < 1)
      v = 1;
    return v;
  }();
  return per_cu * n_cu;
}

bool gemm_quad_pad_even(int prec) {
  static_assert(QuadCfg<SPAMM_BF16, 1>::NP == 1 && QuadCfg<SPAMM_F32, 1>::NP % 2 == 0 &&
                    QuadCfg<SPAMM_BF16X3, 1>::NP % 2 == 0 && QuadCfg<SPAMM_F64, 0>::NP % 2 == 0,
                "only BF16 has one panel per product");
  return prec == SPAMM_BF16;
}

bool gemm_quad_supported(int prec, int bs) {
  return (bs == 64 || bs == 128 || bs == 256) && prec >= SPAMM_F64 && prec <= SPAMM_BF16X3;
}

// Quads take 16 x 16 MFMA tiles in every precision (the 32 x 32 variant
// needs more registers than the pipelined kernel leaves).
template <typename F>
static auto dispatch_quad(int prec, F&& f) {
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  switch (prec) {
    case SPAMM_F64: return f(std::integral_constant<int, SPAMM_F64>{}, I0{});
    case SPAMM_F32: return f(std::integral_constant<int, SPAMM_F32>{}, I1{});
    case SPAMM_BF16: return f(std::integral_constant<int, SPAMM_BF16>{}, I1{});
    default: return f(std::integral_constant<int, SPAMM_BF16X3>{}, I1{});
  }
}

int gemm_quad_max_groups(int prec, int n_cu) {
  return dispatch_quad(prec, [&](auto pc, auto vc) -> int {
    return max_groups_quad<decltype(pc)::value, decltype(vc)::value>(n_cu);
  });
}

template <int P, int V, int RS>
static hipError_t launch_quad_rs(hipStream_t s, const GemmArgs& a) {
  hipLaunchKernelGGL((k_gemm_quad<P, V, RS>), dim3(uint32_t(kXcds * a.kx)), dim3(QuadCfg<P, V, RS>::NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gemm_quad(hipStream_t s, int prec, int bs, const GemmArgs& a) {
  if (!gemm_quad_supported(prec, bs)) return hipErrorInvalidValue;
  return dispatch_quad(prec, [&](auto pc, auto vc) -> hipError_t {
    constexpr int P = decltype(pc)::value, V = decltype(vc)::value;
    switch (bs) {
      case 64: return launch_quad_rs<P, V, 64>(s, a);
      case 128: return launch_quad_rs<P, V, 128>(s, a);
      default: return launch_quad_rs<P, V, 256>(s, a);
    }
  });
}

// ---------------------------------------------------------------- launch

template <int P, int BS, int V, int LS>
static int max_groups(int n_cu) {
  static const int per_cu = [] {  // thread-safe one-time query
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_gemm<P, BS, V, LS>, GemmCfg<P, BS, V, LS>::NT, 0) !=
            hipSuccess ||
        v < 1)
      v = 1;
    return v;
  }();
  return per_cu * n_cu;
}

template <int P, int BS, int V, int LS>
static hipError_t launch_one(hipStream_t s, const GemmArgs& a) {
  hipLaunchKernelGGL((k_gemm<P, BS, V, LS>), dim3(uint32_t(kXcds * a.kx)), dim3(GemmCfg<P, BS, V, LS>::NT), 0, s,
                     a);
  return hipGetLastError();
}

bool gemm_supported(int prec, int bs) {
  if (prec == SPAMM_F64 || prec == SPAMM_F32) return bs == 16 || bs == 32 || bs == 64 || bs == 128 || bs == 256;
  if (prec == SPAMM_BF16 || prec == SPAMM_BF16X3) return bs == 32 || bs == 64 || bs == 128 || bs == 256;
  return false;
}

// Work units per C leaf: one, or four 128 x 128 tiles of a 256 leaf.
int gemm_unit_tiles(int bs) { return bs == 256 ? 4 : 1; }

// Runtime (precision, leaf, variant) -> kernel instance; f receives the
// C tile side and the leaf side (equal below 256).
template <int P, int V, typename F>
static auto with_leaf(int bs, F&& f) {
  using std::integral_constant;
  switch (bs) {
    case 16:
      if constexpr (P == SPAMM_F64 || P == SPAMM_F32) return f(integral_constant<int, 16>{}, integral_constant<int, 16>{});
      else break;
    case 32: return f(integral_constant<int, 32>{}, integral_constant<int, 32>{});
    case 64: return f(integral_constant<int, 64>{}, integral_constant<int, 64>{});
    case 128: return f(integral_constant<int, 128>{}, integral_constant<int, 128>{});
    case 256: return f(integral_constant<int, 128>{}, integral_constant<int, 256>{});
    default: break;
  }
  return f(integral_constant<int, 0>{}, integral_constant<int, 0>{});
}

template <typename F>
static auto dispatch(int prec, int bs, int variant, F&& f) {
  auto go = [&](auto pc, auto vc) {
    return with_leaf<decltype(pc)::value, decltype(vc)::value>(bs, [&](auto tc, auto lc) { return f(pc, tc, vc, lc); });
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  switch (prec) {
    case SPAMM_F64: return go(std::integral_constant<int, SPAMM_F64>{}, I0{});
    case SPAMM_F32:
      return variant ? go(std::integral_constant<int, SPAMM_F32>{}, I1{}) : go(std::integral_constant<int, SPAMM_F32>{}, I0{});
    case SPAMM_BF16:
      return variant ? go(std::integral_constant<int, SPAMM_BF16>{}, I1{}) : go(std::integral_constant<int, SPAMM_BF16>{}, I0{});
    default:
      return variant ? go(std::integral_constant<int, SPAMM_BF16X3>{}, I1{})
                     : go(std::integral_constant<int, SPAMM_BF16X3>{}, I0{});
  }
}

int gemm_max_groups(int prec, int bs, int variant, int n_cu) {
  if (!gemm_supported(prec, bs)) return n_cu;
  return dispatch(prec, bs, variant, [&](auto pc, auto tc, auto vc, auto lc) -> int {
    if constexpr (decltype(tc)::value == 0) return n_cu;
    else return max_groups<decltype(pc)::value, decltype(tc)::value, decltype(vc)::value, decltype(lc)::value>(n_cu);
  });
}

hipError_t launch_gemm(hipStream_t s, int prec, int bs, int variant, const GemmArgs& a) {
  if (!gemm_supported(prec, bs)) return hipErrorInvalidValue;
  return dispatch(prec, bs, variant, [&](auto pc, auto tc, auto vc, auto lc) -> hipError_t {
    if constexpr (decltype(tc)::value == 0) return hipErrorInvalidValue;
    else return launch_one<decltype(pc)::value, decltype(tc)::value, decltype(vc)::value, decltype(lc)::value>(s, a);
  });
}

// ---------------------------------------------------------------- schedule

// Range starts: start[r] = first unit u with prefix[u] >= r * total / nwg
// (prefix is the exclusive scan of the unit costs, prefix[nwu] = total).
__global__ void k_wg_ranges(const int64_t* __restrict__ prefix, int64_t nwu, int nwg, int64_t* __restrict__ start) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > nwg) return;
  const int64_t total = prefix[nwu];
  if (r == 0 || r == nwg) {
    start[r] = r == 0 ? 0 : nwu;
    return;
  }
  const int64_t target = total / nwg * r + (total % nwg) * r / nwg;
  int64_t lo = 0, hi = nwu;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (prefix[mid] >= target) hi = mid;
    else lo = mid + 1;
  }
  start[r] = lo;
}

hipError_t launch_wg_ranges(hipStream_t s, const int64_t* prefix, int64_t nwu, int nwg, int64_t* start) {
  hipLaunchKernelGGL(k_wg_ranges, dim3(uint32_t((nwg + 1 + 255) / 256)), dim3(256), 0, s, prefix, nwu, nwg, start);
  return hipGetLastError();
}

// Leaf norms (leaf level of C's pyramid) and diagonal sums of the units.  A
// leaf split into tiles has its units next to each other (tile 0 first):
// the unit of tile 0 adds the tiles' squared norms, and the diagonal sums of
// the tiles on the leaf's diagonal, in tile order.
__global__ void k_unit_scatter(const ReqDev* __restrict__ reqs, const WorkUnit* __restrict__ wu, int64_t nwu,
                               const double* __restrict__ wn, const double* __restrict__ wt) {
  const int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u >= nwu) return;
  const WorkUnit w = wu[u];
  if (unit_tile(w.cflags) != 0) return;
  const ReqDev& R = reqs[w.req];
  const int nt = R.bs == 256 ? 2 : 1;  // tiles per side
  const uint32_t cm = uint32_t(w.cflags & kUnitMorton);
  double s = 0.0;
  for (int t = 0; t < nt * nt; ++t) s += wn[u + t];
  R.cnorm[level_offset(R.L) + cm] = s;
  uint32_t ci, cj;
  demorton(cm, ci, cj);
  if (ci == cj) {
    double d = 0.0;
    for (int t = 0; t < nt; ++t) d += wt[u + t * nt + t];
    R.trace_part[ci] = d;
  }
}

hipError_t launch_unit_scatter(hipStream_t s, const ReqDev* reqs, const WorkUnit* wu, int64_t nwu, const double* wn,
                               const double* wt) {
  if (nwu == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_scatter, dim3(uint32_t((nwu + 255) / 256)), dim3(256), 0, s, reqs, wu, nwu, wn, wt);
  return hipGetLastError();
}

}  // namespace spamm
