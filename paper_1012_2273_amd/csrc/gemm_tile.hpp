// gemm_tile.hpp -- one output tile of C = op(A) * op(B) on the CDNA4 matrix
// cores (gfx950). Shared by the single-product kernels and the persistent
// grouped kernel.
//
// The product is the one of Hasta and Mutiara, Section 3.1, Algorithm 1:
// every c[i][j] is the sum over p of a[i][p] * b[p][j], with C zeroed first
// (Algorithms 3 and 4). Here the reduction over p is blocked into K-tiles of
// BK and handed to MFMA instructions; the order of the partial sums differs
// from the paper's sequential loop, the set of products does not.
//
// Data path of one workgroup (4 wave64s, 256 threads):
//   HBM/L2 --16-byte vector loads--> VGPR prefetch (tile k+1)
//   VGPR --ds_write--> LDS stage (k+1)&1     (double buffer, one barrier/tile)
//   LDS stage k&1 --ds_read_b128--> operand fragments --> MFMA (AccVGPRs)
//   accumulators --masked stores--> C
//
// LDS layout: both operands are kept "K-contiguous", X[r][0..BK) for the
// r-th row of op(A) or the r-th column of op(B), rows padded by 16 bytes.
// Lane group g = lane/16 of a wave owns the K sub-range [g*BK/4, (g+1)*BK/4)
// of every K-tile and feeds it to the MFMAs in steps of KPL elements; A and
// B use the same mapping, so each MFMA still pairs a[i][p] with b[p][j].
//
// Operand storage in memory (per operand, a template flag):
//   K-contiguous  (A not transposed, or B transposed): vector loads go to LDS
//                 unchanged;
//   MN-contiguous (A transposed, or B not transposed): vector loads along
//                 M (or N) are scattered into the K-contiguous LDS rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace g355 {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

enum Prec : int {
  PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_SPLIT = 3, PREC_SPLIT3 = 4,
  PREC_FSPLIT = 5, PREC_FSPLIT3 = 6,  // split in registers from binary32 tiles
  PREC_LSPLIT = 7, PREC_LSPLIT3 = 8   // split by loader waves from binary32 into LDS planes
};

// Per-precision description of the MFMA used and the element types.
//   E    element type in global memory and LDS (bf16 kept as 16-bit pattern)
//   Op   the per-lane operand of one MFMA
//   Acc  the per-lane accumulator of one 16x16 output block
//   KPL  K elements per lane per MFMA (16x16x4 -> 1, 16x16x32 -> 8)
//   BK   K-tile depth of the small shapes (see bk_of)
//   GRP  rows per lane group in the 16x16 output block: lane l holds column
//        l%16 and rows (q/GRP)*4*GRP + (l/16)*GRP + q%GRP, q = 0..3
//        (binary64: rows 4q + l/16; binary32 accumulators: rows 4(l/16) + q)
//   CVT  bfloat16 terms each binary32 element is split into in registers
//        between the LDS read and the MFMA (0: operands used as loaded)
template <int P> struct Traits;
template <> struct Traits<PREC_F64> {
  using E = double; using Op = double; using Acc = f64x4; using Out = double;
  static constexpr int KPL = 1, BK = 16, PLANES = 1, GRP = 1, CVT = 0;
};
template <> struct Traits<PREC_F32> {
  using E = float; using Op = float; using Acc = f32x4; using Out = float;
  static constexpr int KPL = 1, BK = 16, PLANES = 1, GRP = 4, CVT = 0;
};
template <> struct Traits<PREC_BF16> {
  using E = uint16_t; using Op = u16x8; using Acc = f32x4; using Out = float;
  static constexpr int KPL = 8, BK = 32, PLANES = 1, GRP = 4, CVT = 0;
};
#ifndef G355_SPLIT_BK
#define G355_SPLIT_BK 64
#endif
#ifndef G355_BF16_W8_BK
#define G355_BF16_W8_BK 32
#endif
template <> struct Traits<PREC_SPLIT> {
  using E = uint16_t; using Op = u16x8; using Acc = f32x4; using Out = float;
  static constexpr int KPL = 8, BK = G355_SPLIT_BK, PLANES = 2, GRP = 4, CVT = 0;   // hi and lo planes
};
template <> struct Traits<PREC_SPLIT3> {
  using E = uint16_t; using Op = u16x8; using Acc = f32x4; using Out = float;
  static constexpr int KPL = 8, BK = 32, PLANES = 3, GRP = 4, CVT = 0;   // hi, mid and lo planes
};
// The same two products with the split done per fragment in registers: the
// operands are the binary32 matrices themselves, the K-tile depths and the
// MFMA order are those of the plane products, so the results are the same
// bit for bit.
template <> struct Traits<PREC_FSPLIT> {
  using E = float; using Op = u16x8; using Acc = f32x4; using Out = float;
  static constexpr int KPL = 8, BK = G355_SPLIT_BK, PLANES = 1, GRP = 4, CVT = 2;
};
template <> struct Traits<PREC_FSPLIT3> {
  using E = float; using Op = u16x8; using Acc = f32x4; using Out = float;
  static constexpr int KPL = 8, BK = 32, PLANES = 1, GRP = 4, CVT = 3;
};

// The same products once more with the planes made inside the workgroup:
// loader waves read binary32 tiles of A and B into registers, split them and
// write the bfloat16 planes into the LDS ring, where the compute waves read
// them exactly as the plane products read transferred planes (A K-contiguous,
// B N-contiguous): the same bits again, without the planes in device memory.
template <> struct Traits<PREC_LSPLIT> {
  using E = uint16_t; using Op = u16x8; using Acc = f32x4; using Out = float;
  static constexpr int KPL = 8, BK = G355_SPLIT_BK, PLANES = 2, GRP = 4, CVT = 0;
};
template <> struct Traits<PREC_LSPLIT3> {
  using E = uint16_t; using Op = u16x8; using Acc = f32x4; using Out = float;
  static constexpr int KPL = 8, BK = 32, PLANES = 3, GRP = 4, CVT = 0;
};
// Planes the loader waves make from binary32 operands (0: operands arrive
// as they are used).
template <int P> __host__ __device__ constexpr int lcv_of() {
  return P == PREC_LSPLIT ? 2 : P == PREC_LSPLIT3 ? 3 : 0;
}

// x split into NP bfloat16 terms, each rounded to nearest even from what the
// earlier terms leave (Dekker-style splitting): t0 = bf16(x), t1 = bf16(x -
// t0), t2 = bf16(x - t0 - t1). Every subtraction is exact in binary32 (the
// remainder fits in 24 bits), so the terms are unique. Used by the split
// step and by the in-register split of the fused products alike.
template <int NP> __device__ __forceinline__ void split_x(float x, uint16_t (&o)[NP]) {
  float r = x;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const __bf16 b = (__bf16)r;
    o[p] = __builtin_bit_cast(uint16_t, b);
    if (p + 1 < NP) r = r - (float)b;
  }
}

// The products of a split precision, as (A plane, B plane) pairs in the
// order they are accumulated: smallest terms first, so that the large ones
// are added to an accumulator that already holds the small ones. Plane 0 is
// hi, 1 lo (two planes) or mid, 2 lo (three planes). Two planes: lo*hi,
// hi*lo, hi*hi (lo*lo dropped). Three planes: lo*hi, hi*lo, mid*mid,
// mid*hi, hi*mid, hi*hi (mid*lo, lo*mid, lo*lo dropped).
template <int PL> struct Terms;
template <> struct Terms<1> {
  static constexpr int N = 1;
  static constexpr int a[1] = {0}, b[1] = {0};
};
template <> struct Terms<2> {
  static constexpr int N = 3;
  static constexpr int a[3] = {1, 0, 0}, b[3] = {0, 1, 0};
};
template <> struct Terms<3> {
  static constexpr int N = 6;
  static constexpr int a[6] = {2, 0, 1, 1, 0, 0}, b[6] = {0, 2, 1, 0, 1, 0};
};

__device__ __forceinline__ void mfma(f64x4 &acc, double a, double b) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}
__device__ __forceinline__ void mfma(f32x4 &acc, float a, float b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}
__device__ __forceinline__ void mfma(f32x4 &acc, u16x8 a, u16x8 b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
__device__ __forceinline__ void mfma(f32x16 &acc, u16x8 a, u16x8 b) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
}

template <typename T, int V> struct alignas(sizeof(T) * V) VecT { T e[V]; };

// Arguments of one product. For PREC_SPLIT, A/B are the hi planes and
// A2/B2 the lo planes; for PREC_SPLIT3, A/B hi, A2/B2 mid and A3/B3 lo (all
// planes of an operand share its leading dimension).
struct GemmArgs {
  int64_t M, N, K;
  const void *A; int64_t lda;
  const void *B; int64_t ldb;
  const void *A2; const void *B2;
  void *C; int64_t ldc;
  const void *A3 = nullptr; const void *B3 = nullptr;
};

// Tile shape: BM x BN outputs per workgroup, WM x WN wave positions (64
// lanes each), KS waves per position splitting every K-tile between them
// (their partial sums are added through LDS at the end of the tile); KB > 0
// fixes the K-tile depth of the direct-to-LDS path (else bk_of's rule);
// LDW > 0 adds that many loader waves, which issue every operand transfer of
// the direct-to-LDS path and no MFMA (the other waves then only compute).
template <int BM_, int BN_, int WM_, int WN_, int KS_ = 1, int KB_ = 0, int LDW_ = 0> struct Shape {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KS = KS_, KB = KB_, LDW = LDW_;
  static constexpr int NC = 64 * WM * WN * KS;   // compute threads
  static constexpr int NT = NC + 64 * LDW;
  static constexpr int WTM = BM / WM, WTN = BN / WN;   // per-wave tile
  static constexpr int FM = WTM / 16, FN = WTN / 16;   // 16x16 blocks per wave
  static_assert(FM >= 1 && FN >= 1 && WTM % 16 == 0 && WTN % 16 == 0, "bad shape");
};

// K-tile depth of a (precision, shape) pair on the direct-to-LDS path:
// binary64 tiles of 128 x 128 outputs with 8 waves (one workgroup per CU)
// take 32-deep K-tiles (twice the MFMA work per barrier), and so does the
// 4-wave 32 x 32 and 64 x 64 tiles, which run one or two workgroups per CU
// at the sizes they serve and wait on each K-tile's transfers there (half
// as many round trips: N = 500 15.6 -> 12.8 us, N = 700 27.3 -> 23.6 on
// 32 x 32; N = 1400 110.5 -> 98.5, N = 3600 +2% on 64 x 64, N = 1500 and
// 1700 0.7% and 1.7% slower); the others keep 16 so that two or more
// workgroups fit in LDS. binary32 takes 16 unless a
// 16-deep K-tile of A or B is fewer 1 KiB transfers than the shape has
// waves (the 8-wave 128 x 64 and 64 x 64 shapes), then 32, and 32 on the
// 4-wave 128 x 128 tile (two workgroups of 64 KiB per CU: 131.8 against
// 124.2 TFLOP/s at N = 4096 with 16-deep K-tiles and three workgroups). A
// shape's KB overrides the rule. The register path uses Traits<P>::BK.
template <int P, class S> __host__ __device__ constexpr int bk_of() {
  if constexpr (S::KB > 0) {
    return S::KB;
  } else if constexpr (P == PREC_F64) {
    return (S::BM * S::BN >= 128 * 128 && S::NT >= 512) || (S::BM * S::BN <= 64 * 64 && S::KS == 1 && S::NT == 256)
               ? 32 : 16;
  } else if constexpr ((P == PREC_F32 || P == PREC_BF16) && S::BM * S::BN <= 32 * 32 &&
                       S::KS == 1 && S::NT == 256) {
    // the 4-wave 32 x 32 tile of the small products, for the same reason as
    // binary64's: binary32 N = 500 9.4 -> 8.1-8.4 us, N = 700 16.0 -> 13.6;
    // bf16 N = 600 10.1 -> 7.8-8.2, level elsewhere
    return 64;
  } else if constexpr (P == PREC_F32) {
    constexpr int waves = S::NT / 64;
    constexpr bool even16 = (S::BM * 16 * 4 / 1024) % waves == 0 && (S::BN * 16 * 4 / 1024) % waves == 0;
    constexpr bool big4 = S::NT == 256 && S::BM * S::BN >= 128 * 128;
    return even16 && !big4 ? 16 : 32;
  } else if constexpr (P == PREC_BF16 && S::KS > 1) {
    return 64;
  } else if constexpr (P == PREC_BF16 && S::NT >= 512 && S::BM * S::BN == 128 * 128) {
    return G355_BF16_W8_BK;
  } else {
    return Traits<P>::BK;
  }
}

// A K split needs every wave's share of a K-tile to hold whole MFMA steps.
template <int P, class S> __host__ __device__ constexpr bool shape_ok() {
  constexpr int KG = Traits<P>::BK / 4;
  return KG % S::KS == 0 && (KG / S::KS) % Traits<P>::KPL == 0;
}

template <int P> __host__ __device__ constexpr int lds_pad() {
  return 16 / (int)sizeof(typename Traits<P>::E);       // 16 bytes per row
}
template <int P, class S> __host__ __device__ constexpr int lds_bytes() {
  using T = Traits<P>;
  constexpr int stages =
      2 * T::PLANES * (S::BM + S::BN) * (T::BK + lds_pad<P>()) * (int)sizeof(typename T::E);
  // K-split reduction: one wave column (BM x WTN accumulators) at a time
  constexpr int red = S::KS > 1 ? S::BM * S::WTN * (int)sizeof(typename T::Acc) / 4 : 0;
  return stages > red ? stages : red;
}

// Buffer resource over `base` for raw buffer loads (CDNA: 32-bit data
// format in word 3). Offsets at or above kOob read as zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, 0x7fffffff,
                                           0x00020000);
}
constexpr uint32_t kOob = 0x80000000u;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int BYTES> struct RawT;
template <> struct RawT<16> { using T = u32x4; };
template <> struct RawT<8> { using T = u32x2; };
template <> struct RawT<4> { using T = uint32_t; };
template <> struct RawT<2> { using T = uint16_t; };

template <int BYTES>
__device__ __forceinline__ typename RawT<BYTES>::T raw_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (BYTES == 16) return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  else if constexpr (BYTES == 8) return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  else if constexpr (BYTES == 4) return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  else return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
}

// Global -> VGPR -> LDS mover for one operand plane of R rows x BK.
//   KC = true : element (r, p) at base[(r0 + r) * ld + k0 + p]
//   KC = false: element (r, p) at base[(k0 + p) * ld + r0 + r]
// Each thread moves whole vectors of V = VW / sizeof(E) elements (VW = 16 or
// 8 bytes; one element for VW = 0) along the contiguous direction. The host
// enables V > 1 only when every vector is entirely inside or entirely outside
// the matrix (VW-byte aligned base and ld, and the contiguous extent a
// multiple of V); an outside vector gets the offset kOob
// and the buffer unit returns zeros, so the tile edges need no branches.
// Offsets are 32-bit byte offsets from the K-tile's base: R * ld * sizeof(E)
// must stay below 2^31 (the host checks).
template <typename E, int R, int BK, int NT, bool KC, int VW>
struct Mover {
  static constexpr int V = VW > (int)sizeof(E) ? VW / (int)sizeof(E) : 1;
  static constexpr int NVEC = R * BK / V;
  static constexpr int PER = (NVEC + NT - 1) / NT;
  static constexpr bool FULL = (NVEC % NT) == 0;
  static constexpr int LDW = BK + 16 / (int)sizeof(E);   // padded LDS row
  using Raw = typename RawT<V * (int)sizeof(E)>::T;

  Raw buf[PER];
  uint32_t off[PER];    // byte offset of the slot within a K-tile
  bool rok[PER];        // the slot's row (M or N index) is inside the matrix

  __device__ __forceinline__ static void slot(int i, int tid, int &r, int &p) {
    const int v = tid + i * NT;
    if constexpr (KC) { r = v / (BK / V); p = (v % (BK / V)) * V; }
    else              { p = v / (R / V);  r = (v % (R / V)) * V; }
  }

  __device__ __forceinline__ void init(int64_t ld, int64_t r0, int64_t rtot, int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      int r, p;
      slot(i, tid, r, p);
      const bool live = FULL || (tid + i * NT < NVEC);
      rok[i] = live && (r0 + r < rtot);
      if constexpr (KC) off[i] = (uint32_t)(((int64_t)r * ld + p) * (int64_t)sizeof(E));
      else              off[i] = (uint32_t)(((int64_t)p * ld + r) * (int64_t)sizeof(E));
    }
  }

  // tile_base: element (r0, k0) for KC, (k0, r0) otherwise.
  __device__ __forceinline__ void load(const E *tile_base, int64_t k0, int64_t K, int tid) {
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(tile_base);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      int r, p;
      slot(i, tid, r, p);
      const bool ok = rok[i] && (k0 + p < K);
      buf[i] = raw_load<V * (int)sizeof(E)>(rs, ok ? off[i] : kOob);
    }
  }

  __device__ __forceinline__ void store(E *lds, int tid) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (!FULL && tid + i * NT >= NVEC) continue;
      int r, p;
      slot(i, tid, r, p);
      if constexpr (KC) {
        *reinterpret_cast<Raw *>(lds + r * LDW + p) = buf[i];
      } else {
        const VecT<E, V> v = __builtin_bit_cast(VecT<E, V>, buf[i]);
#pragma unroll
        for (int e = 0; e < V; ++e) lds[(r + e) * LDW + p] = v.e[e];
      }
    }
  }
};

// Compute one BM x BN tile of C at (m0, n0). TA: op(A) = A^T (A stored
// K x M); TB: op(B) = B^T (B stored N x K). VW: vector loads of VW bytes
// allowed (16 or 8; 0: element loads).
//
// Schedule of one K-tile for one wave (U read units of the wave's K range):
//   issue global loads of K-tile t+1 into VGPRs
//   for each unit u < U-1: LDS reads of unit u+1 | MFMAs of unit u
//   MFMAs of the first half of the last unit's blocks
//   VGPRs -> LDS stage of t+1; barrier; LDS reads of unit 0 of t+1
//   MFMAs of the second half of the last unit's blocks
// so the global-load latency is covered by the MFMAs before the store, and
// the barrier and the first LDS reads of the next tile by the last half.
template <int P, class S, bool TA, bool TB, int VW>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int64_t m0, int64_t n0,
                                          char *smem) {
  using T = Traits<P>;
  using E = typename T::E;
  using Op = typename T::Op;
  using Acc = typename T::Acc;
  using Out = typename T::Out;
  constexpr int BK = T::BK, KPL = T::KPL, PL = T::PLANES, KS = S::KS;
  constexpr int LDW = BK + lds_pad<P>();
  constexpr int KG = BK / 4;             // K elements per lane group per tile
  constexpr int KW = KG / KS;            // ... owned by one wave of a K split
  constexpr int RU = (16 / (int)sizeof(E)) < KW ? (16 / (int)sizeof(E)) : KW;  // per read
  constexpr int U = KW / RU;             // read units per tile per wave
  constexpr int SPU = RU / KPL;          // MFMA steps per read unit
  static_assert(KG % KS == 0 && KW % RU == 0 && RU % KPL == 0, "bad K split");
  constexpr int NT = S::NT;
  constexpr int A_ELEMS = S::BM * LDW, B_ELEMS = S::BN * LDW;
  constexpr int STAGE = PL * (A_ELEMS + B_ELEMS);
  constexpr int NB = S::FM * S::FN;      // 16x16 blocks per wave
  constexpr int NB1 = NB / 2;            // blocks before the barrier in the last unit

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wpos = wave % (S::WM * S::WN), kh = wave / (S::WM * S::WN);
  const int wm = wpos % S::WM, wn = wpos / S::WM;
  const int lr = lane & 15, lgp = lane >> 4;

  E *lds = reinterpret_cast<E *>(smem);
  const E *Ap[3] = {reinterpret_cast<const E *>(g.A), reinterpret_cast<const E *>(g.A2),
                    reinterpret_cast<const E *>(g.A3)};
  const E *Bp[3] = {reinterpret_cast<const E *>(g.B), reinterpret_cast<const E *>(g.B2),
                    reinterpret_cast<const E *>(g.B3)};

  // 8-byte vectors only along K: an MN-contiguous vector is stored to the
  // K-major LDS tile one element per row, and four rows per lane put 16
  // lanes of a 2-byte store on one bank (bf16 N = 4300: 164 against 296
  // TFLOP/s with element loads)
  constexpr int VWA = (VW == 8 && TA) ? 0 : VW, VWB = (VW == 8 && !TB) ? 0 : VW;
  Mover<E, S::BM, BK, NT, !TA, VWA> ma[PL];
  Mover<E, S::BN, BK, NT, TB, VWB> mb[PL];

  Acc acc[S::FM][S::FN];
#pragma unroll
  for (int i = 0; i < S::FM; ++i)
#pragma unroll
    for (int j = 0; j < S::FN; ++j) acc[i][j] = Acc{};

  const int64_t KT = (g.K + BK - 1) / BK;

#pragma unroll
  for (int pl = 0; pl < PL; ++pl) {
    ma[pl].init(g.lda, m0, g.M, tid);
    mb[pl].init(g.ldb, n0, g.N, tid);
  }
  auto load_tile = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) {
      const E *ta = TA ? Ap[pl] + k0 * g.lda + m0 : Ap[pl] + m0 * g.lda + k0;
      const E *tb = TB ? Bp[pl] + n0 * g.ldb + k0 : Bp[pl] + k0 * g.ldb + n0;
      ma[pl].load(ta, k0, g.K, tid);
      mb[pl].load(tb, k0, g.K, tid);
    }
  };
  auto store_tile = [&](int stage) {
    E *st = lds + stage * STAGE;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) {
      ma[pl].store(st + pl * A_ELEMS, tid);
      mb[pl].store(st + PL * A_ELEMS + pl * B_ELEMS, tid);
    }
  };

  // Fragments of one read unit: RU consecutive K elements per lane for each
  // block row (A) and block column (B); double-buffered across units.
  using Unit = VecT<E, RU>;
  Unit fa[2][PL][S::FM], fb[2][PL][S::FN];
  auto read_unit = [&](int stage, int u, auto buf_tag) {
    constexpr int b = decltype(buf_tag)::value;
    const E *st = lds + stage * STAGE;
    const int koff = lgp * KG + kh * KW + u * RU;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) {
#pragma unroll
      for (int i = 0; i < S::FM; ++i)
        fa[b][pl][i] = *reinterpret_cast<const Unit *>(
            st + pl * A_ELEMS + (wm * S::WTM + i * 16 + lr) * LDW + koff);
#pragma unroll
      for (int j = 0; j < S::FN; ++j)
        fb[b][pl][j] = *reinterpret_cast<const Unit *>(
            st + PL * A_ELEMS + pl * B_ELEMS + (wn * S::WTN + j * 16 + lr) * LDW + koff);
    }
  };
  auto op_of = [](const Unit &u, int step) {
    return *reinterpret_cast<const Op *>(&u.e[step * KPL]);
  };
  // MFMAs of blocks [lo, hi) of a unit, every step of the unit.
  auto mma_unit = [&](auto buf_tag, auto lo_tag, auto hi_tag) {
    constexpr int b = decltype(buf_tag)::value;
    constexpr int lo = decltype(lo_tag)::value, hi = decltype(hi_tag)::value;
    using TM = Terms<PL>;
#pragma unroll
    for (int st = 0; st < SPU; ++st) {
      // the terms of a split precision, smallest first, into one accumulator
#pragma unroll
      for (int t = 0; t < TM::N; ++t) {
#pragma unroll
        for (int x = lo; x < hi; ++x)
          mfma(acc[x / S::FN][x % S::FN], op_of(fa[b][TM::a[t]][x / S::FN], st),
               op_of(fb[b][TM::b[t]][x % S::FN], st));
      }
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using INB1 = std::integral_constant<int, NB1>;
  using INB = std::integral_constant<int, NB>;

  // One K-tile; P0 is the fragment buffer of its unit 0 (static, so the
  // fragments stay in registers; with an odd U the parity alternates and the
  // loop below is unrolled by two).
  auto ktile = [&](auto p0_tag, int64_t kt) {
    constexpr int P0 = decltype(p0_tag)::value;
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < KT;
    if (more) load_tile(kt + 1);
    [&]<int... u>(std::integer_sequence<int, u...>) {
      ((read_unit(cur, u + 1, std::integral_constant<int, (P0 + u + 1) & 1>{}),
        mma_unit(std::integral_constant<int, (P0 + u) & 1>{}, I0{}, INB{})), ...);
    }(std::make_integer_sequence<int, U - 1>{});
    constexpr int PL_ = (P0 + U - 1) & 1;
    mma_unit(std::integral_constant<int, PL_>{}, I0{}, INB1{});
    if (more) store_tile(cur ^ 1);
    __syncthreads();
    if (more) read_unit(cur ^ 1, 0, std::integral_constant<int, (P0 + U) & 1>{});
    mma_unit(std::integral_constant<int, PL_>{}, INB1{}, INB{});
  };

  if (KT > 0) {
    load_tile(0);
    store_tile(0);
    __syncthreads();
    read_unit(0, 0, I0{});
    if constexpr (U % 2 == 0) {
      for (int64_t kt = 0; kt < KT; ++kt) ktile(I0{}, kt);
    } else {
      for (int64_t kt = 0; kt < KT; kt += 2) {
        ktile(I0{}, kt);
        if (kt + 1 < KT) ktile(std::integral_constant<int, 1>{}, kt + 1);
      }
    }
  }

  // K split: waves kh > 0 hand their partial sums to kh = 0 through LDS, one
  // wave column at a time (the operand stages are free after the last barrier).
  if constexpr (KS > 1) {
    using AE = std::remove_reference_t<decltype(acc[0][0][0])>;
    AE *red = reinterpret_cast<AE *>(smem);
#pragma unroll 1
    for (int col = 0; col < S::WN; ++col) {
#pragma unroll 1
      for (int h = 1; h < KS; ++h) {
        if (wn == col && kh == h) {
#pragma unroll
          for (int i = 0; i < S::FM; ++i)
#pragma unroll
            for (int j = 0; j < S::FN; ++j)
#pragma unroll
              for (int q = 0; q < 4; ++q)
                red[(((wm * S::FM + i) * S::FN + j) * 4 + q) * 64 + lane] = acc[i][j][q];
        }
        __syncthreads();
        if (wn == col && kh == 0) {
#pragma unroll
          for (int i = 0; i < S::FM; ++i)
#pragma unroll
            for (int j = 0; j < S::FN; ++j)
#pragma unroll
              for (int q = 0; q < 4; ++q)
                acc[i][j][q] += red[(((wm * S::FM + i) * S::FN + j) * 4 + q) * 64 + lane];
        }
        __syncthreads();
      }
    }
    if (kh != 0) return;
  }

  // Epilogue: lane holds column lane%16 of each 16x16 block and the four
  // rows given by the precision's output grouping (Traits::GRP).
  constexpr int GRP = T::GRP;
  Out *C = reinterpret_cast<Out *>(g.C);
#pragma unroll
  for (int i = 0; i < S::FM; ++i) {
#pragma unroll
    for (int j = 0; j < S::FN; ++j) {
      const int64_t col = n0 + wn * S::WTN + j * 16 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = m0 + wm * S::WTM + i * 16 + (q / GRP) * 4 * GRP + lgp * GRP + q % GRP;
        if (row < g.M && col < g.N) C[row * g.ldc + col] = (Out)acc[i][j][q];
      }
    }
  }
}

// Map a linear workgroup id onto a tile so that the workgroups one XCD
// receives (ids x, x+8, x+16, ... go to XCD x) form one contiguous range of
// a grouped raster: tiles that share rows of A or columns of B then share an
// L2. `group_m` rows of tiles are walked column by column.
__device__ __forceinline__ void tile_of(int wg, int nwg, int tiles_m, int tiles_n,
                                        int group_m, int &tm, int &tn) {
  constexpr int XCD = 8;
  const int q = nwg / XCD, rem = nwg % XCD;
  const int x = wg % XCD, j = wg / XCD;
  const int t = x * q + (x < rem ? x : rem) + j;
  const int per_group = group_m * tiles_n;
  const int grp = t / per_group;
  const int first_m = grp * group_m;
  const int gsz = (tiles_m - first_m) < group_m ? (tiles_m - first_m) : group_m;
  const int in = t - grp * per_group;
  tm = first_m + in % gsz;
  tn = in / gsz;
}

}  // namespace g355
