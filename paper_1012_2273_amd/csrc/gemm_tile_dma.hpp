// gemm_tile_dma.hpp -- the tile routine with direct-to-LDS operand loads.
//
// Same product and MFMA mapping as gemm_tile (Hasta and Mutiara, Section 3.1,
// Algorithm 1, reduction blocked over K-tiles), different data movement:
// operands go HBM/L2 -> LDS with `buffer_load_dwordx4 ... lds` (no VGPR
// staging), into a ring of two to eight LDS stages, several K-tiles ahead
// of the MFMAs. Waits are explicit: every loader wave (all waves, or the first
// half or quarter where a K-tile's transfers do not divide evenly) issues the
// same number of 16-byte transfers per K-tile, so `s_waitcnt vmcnt(n)` with
// n = one tile's count retires exactly the tile about to be read; a barrier
// then makes all waves' transfers visible.
//
// LDS layouts (one transfer instruction fills 1 KiB: lane l -> base + 16 l):
//  * K-contiguous operand (A not transposed, B transposed): rows of BK
//    elements, 16-byte chunks XOR-swizzled per row (chunk c of row r holds
//    global chunk c ^ swz(r)) so that sixteen lanes reading the same K
//    offset of sixteen rows hit distinct banks.
//  * MN-contiguous operand (A transposed, B not transposed): rows of R
//    elements, one per k, as in memory. 4- and 8-byte elements: a lane's
//    MFMA operand is one element, read per step from row k. 16-bit
//    elements: 16-byte chunks XOR-swizzled per row in pairs (32-byte
//    column blocks stay whole), read with the transposing LDS read
//    (ds_read_b64_tr_b16), which hands each lane four consecutive k of one
//    column: within a group of 16 lanes, lane 4a + e receives element e of
//    the 8 bytes addressed by lanes a, a + 4, a + 8, a + 12, so lanes
//    a + 4j address row k + j at column 4a of the group's 16 columns.
#pragma once

#include "gemm_tile.hpp"

namespace g355 {


typedef short s16x4 __attribute__((ext_vector_type(4)));

// s_waitcnt encodings (gfx9): vmcnt in bits [3:0] and [15:14], expcnt [6:4],
// lgkmcnt [11:8]; unused counters at their maximum.
template <int VM> __device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(VM >= 0 && VM < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((VM & 0xF) | ((VM >> 4) << 14) | (0x7 << 4) | (0x0 << 8));
}
// One 16-byte-per-lane transfer HBM/L2 -> LDS: lane l's 16 bytes at buffer
// offset `voff` land at LDS byte address lds_base + 16 l (an offset at or
// above the buffer's record count reads as zeros). Issued from inline
// assembly so that the compiler does not add a wait for all outstanding
// transfers before every later LDS read (it cannot tell the ring stages
// apart); the kernel retires transfers itself with wait_vm_lgkm0. The
// instruction writes no VGPR; VMEM loads retire in order, so transfers the
// compiler does not know about only make its own vmcnt waits stricter.
typedef unsigned int srd_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ srd_t make_srd(const void *base) {
  const uint64_t a = (uint64_t)(uintptr_t)base;
  srd_t r;
  r.x = __builtin_amdgcn_readfirstlane((uint32_t)a);
  r.y = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32) & 0xFFFFu);
  r.z = 0x7fffffffu;      // record count (bytes)
  r.w = 0x00020000u;      // 32-bit data format (CDNA)
  return r;
}
__device__ __forceinline__ void lds_dma16(srd_t srd, uint32_t voff, uint32_t lds_base) {
  asm volatile(
      "s_mov_b32 m0, %2\n\t"
      "s_nop 0\n\t"
      "buffer_load_dwordx4 %0, %1, 0 offen lds"
      :
      : "v"(voff), "s"(srd), "s"(lds_base)
      : "memory", "m0");
}
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char *)p;
}

// Workgroup barrier without the memory fence of __syncthreads (whose release
// would wait for every outstanding LDS transfer); the signal fences keep the
// compiler from moving memory operations across it.
__device__ __forceinline__ void raw_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// One operand plane of one K-tile: R rows (M or N) x BK. LG: K rows
// between the lane groups of one LDS read, MBW: lanes per lane group (the
// MFMA block width; both set the MN layout swizzle).
template <typename E, int R, int BK, int NT, bool KC, int LG, int MBW = 16, bool FLAT = false>
struct DmaOp {
  static constexpr int ES = (int)sizeof(E);
  static constexpr int V = 16 / ES;                  // elements per chunk
  static constexpr int RB = KC ? BK * ES : R * ES;   // bytes per LDS row
  static constexpr int NROWS = KC ? R : BK;
  static constexpr int CPR = RB / 16;                // chunks per row
  static constexpr int CHUNKS = NROWS * CPR;
  static constexpr int NI = CHUNKS / 64;             // transfers per tile
  static constexpr int NW = NT / 64;
  static constexpr int PERW = NI / NW;               // transfers per wave per tile
  static constexpr int BYTES = CHUNKS * 16;
  static constexpr bool TR = !KC && ES == 2;         // transposing reads
  static constexpr bool OK = (RB % 16 == 0) && (CHUNKS % 64 == 0) && (NI % NW == 0) &&
                             (PERW >= 1) && (KC || ES >= 4 || (TR && CPR % 2 == 0)) &&
                             (!KC || RB <= 256) && (KC || (CPR & (CPR - 1)) == 0) && LG >= 1;

  uint32_t off[PERW > 0 ? PERW : 1];
  uint32_t offr[PERW > 0 ? PERW : 1];  // off, or kOob outside the matrix's M/N extent
  int32_t kk[PERW > 0 ? PERW : 1];   // K index of the chunk (first element)
  bool rok[PERW > 0 ? PERW : 1];     // M/N index inside the matrix

  __device__ __forceinline__ static int swz(int r) { return ((r * RB) >> 8) % CPR; }
  // MN rows. 16-bit elements: rows k .. k+3 of one transposing read put
  // their column blocks (32 bytes for 16-wide MFMA blocks, 64 for 32-wide)
  // in four different bank groups.
  // 4- and 8-byte elements: the 64 / MBW lane groups of a read take rows LG
  // apart, MBW consecutive elements each; moving row k's chunks by
  // (k / LG) % (64 / MBW) such spans puts the groups on different banks.
  // FLAT: rows read 16 bytes per lane (the interleaved reads below), each
  // lane group a whole 256-byte span: no swizzle (measured: ds_read_b128
  // runs at full rate when lane groups 0/1 and 2/3 take their chunks in the
  // same order, ~20% slower when group 1's order differs from group 0's).
  __device__ __forceinline__ static int swzm(int r) {
    if constexpr (KC) return 0;
    else if constexpr (TR) {
      // a half-wave's transposing read takes MBW columns (MBW * 2 bytes) of
      // each of four rows: shift row k by (k % 4) such spans
      constexpr int SPAN = MBW * ES / 16;
      if constexpr (CPR >= 4 * SPAN) return SPAN * (r % 4);
      else if constexpr (CPR >= 8) return 2 * (r % 4);
      else if constexpr (CPR >= 4) return 2 * (r % 2);
      else return 0;
    } else if constexpr (FLAT) {
      return 0;
    } else {
      constexpr int NGR = 64 / MBW, SPAN = MBW * ES / 16;
      return (((r / LG) & (NGR - 1)) * SPAN) & (CPR - 1);
    }
  }

  __device__ __forceinline__ void init(int64_t ld, int64_t r0, int64_t rtot, int wave, int lane) {
#pragma unroll
    for (int j = 0; j < PERW; ++j) {
      const int q = (wave + j * NW) * 64 + lane;
      const int r = q / CPR, c = q % CPR;
      if constexpr (KC) {
        const int k = (c ^ swz(r)) * V;
        off[j] = (uint32_t)(((int64_t)r * ld + k) * ES);
        kk[j] = k;
        rok[j] = r0 + r < rtot;
      } else {
        const int m = (c ^ swzm(r)) * V;
        off[j] = (uint32_t)(((int64_t)r * ld + m) * ES);
        kk[j] = r;
        rok[j] = r0 + m < rtot;
      }
      offr[j] = rok[j] ? off[j] : kOob;
    }
  }

  // tile_base: element (r0, k0) for KC, (k0, r0) otherwise.
  __device__ __forceinline__ void issue(const E *tile_base, int64_t k0, int64_t K, char *region,
                                        int wave) const {
    const srd_t srd = make_srd(tile_base);
    const uint32_t base = lds_addr(region);
#pragma unroll
    for (int j = 0; j < PERW; ++j) {
      const bool ok = rok[j] && (k0 + kk[j] < K);
      const uint32_t dst = __builtin_amdgcn_readfirstlane(base + (uint32_t)(wave + j * NW) * 1024u);
      lds_dma16(srd, ok ? off[j] : kOob, dst);
    }
  }

  // Transfer j of this wave for the K-tile at tile_base (see issue()).
  // krem = K - k0 clamped to int32 (the same on every lane); wave must be
  // wave-uniform (an SGPR value), which keeps the LDS destination scalar
  // arithmetic. offr holds the offset with the M/N edge already applied.
  __device__ __forceinline__ void issue_one(int j, const srd_t &srd, int32_t krem, uint32_t base,
                                            int wave) const {
    const uint32_t dst = base + (uint32_t)(wave + j * NW) * 1024u;
    const uint32_t voff = kk[j] < krem ? offr[j] : kOob;
    __builtin_amdgcn_sched_barrier(0);
    lds_dma16(srd, voff, dst);
    __builtin_amdgcn_sched_barrier(0);
  }

  // RU consecutive K elements (K offset koff, a multiple of RU) of LDS row
  // `row` (KC) or column `row` (MN). For TR the 16 lanes of a group must
  // ask for 16 consecutive columns starting at a multiple of 16, lane i for
  // column start + i, all at the same koff. KC reads of more than one
  // chunk read each chunk at its own swizzled place.
  template <int RU>
  __device__ __forceinline__ static VecT<E, RU> read(const char *region, int row, int koff) {
    VecT<E, RU> v;
    if constexpr (KC && RU > V) {
      static_assert(RU % V == 0, "whole chunks");
      using Chunk = VecT<E, V>;
#pragma unroll
      for (int h = 0; h < RU / V; ++h) {
        const Chunk c = *reinterpret_cast<const Chunk *>(
            region + row * RB + (((koff / V + h) ^ swz(row)) * 16));
#pragma unroll
        for (int e = 0; e < V; ++e) v.e[h * V + e] = c.e[e];
      }
    } else if constexpr (KC) {
      const int c = koff / V, e0 = koff % V;
      v = *reinterpret_cast<const VecT<E, RU> *>(region + row * RB + ((c ^ swz(row)) * 16) + e0 * ES);
    } else if constexpr (TR) {
      static_assert(RU % 4 == 0, "a transposing read delivers four K elements");
      const int l16 = (int)(threadIdx.x & 15);
      const int col = row - l16 + 4 * (l16 & 3);      // the 8 bytes this lane addresses
      const int cc = col / V, ce = col % V;
#pragma unroll
      for (int h = 0; h < RU / 4; ++h) {
        const int k = koff + 4 * h + (l16 >> 2);
        const char *p = region + k * RB + ((cc ^ swzm(k)) * 16) + ce * ES;
        const s16x4 t = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (__attribute__((address_space(3))) s16x4 *)(p));
        // whole 8 bytes at once: element-wise 16-bit inserts made the
        // compiler wait for each read right after issuing it
        __builtin_memcpy(&v.e[4 * h], &t, 8);
      }
    } else {
      const int cc = row / V, ce = row % V;
#pragma unroll
      for (int e = 0; e < RU; ++e) {
        const int k = koff + e;
        v.e[e] = *reinterpret_cast<const E *>(region + k * RB + ((cc ^ swzm(k)) * 16) + ce * ES);
      }
    }
    return v;
  }

  // MN layout: IL consecutive elements (M or N index `row`, a multiple of
  // IL, IL dividing the 16-byte chunk) of K row k, one LDS read.
  template <int IL>
  __device__ __forceinline__ static VecT<E, IL> read_row(const char *region, int row, int k) {
    static_assert(!KC && !TR && V % IL == 0, "MN rows of 4- or 8-byte elements");
    return *reinterpret_cast<const VecT<E, IL> *>(region + k * RB + (((row / V) ^ swzm(k)) * 16) +
                                                   (row % V) * ES);
  }
};

// MFMA block geometry on this path: the 16-bit precisions use 32 x 32 x 16
// blocks (two lane groups of 32, sixteen binary32 accumulators per lane)
// when the wave tile is a multiple of 32 both ways, else 16 x 16 blocks.
//   lane l: block row/column l % MB, lane group l / MB; output register v
//   of lane group g holds row (v / GRP) * (LGN * GRP) + g * GRP + v % GRP.
template <int P, class S> struct Geom {
  static constexpr bool BIG = Traits<P>::KPL == 8 && S::WTM % 32 == 0 && S::WTN % 32 == 0;
  static constexpr int MB = BIG ? 32 : 16;
  static constexpr int LGN = 64 / MB;
  static constexpr int NR = MB * MB / 64;
  static constexpr int FM = S::WTM / MB, FN = S::WTN / MB;
  static constexpr int KG = bk_of<P, S>() / LGN;    // K elements per lane group per tile
  using Acc = typename std::conditional<BIG, f32x16, typename Traits<P>::Acc>::type;
  static constexpr bool OK = KG % S::KS == 0 && (KG / S::KS) % Traits<P>::KPL == 0 &&
                             FM >= 1 && FN >= 1;
};

// LDS budget of the ring on the 16-bit precisions: 48 KiB keeps three
// workgroups of a 128 x 128 bf16 tile on a CU, which measured faster than
// deeper rings at one or two workgroups per CU (N = 2000 ... 8192).
#ifndef G355_RING16_KB
#define G355_RING16_KB 48
#endif
constexpr int kRing16 = G355_RING16_KB * 1024;
#ifndef G355_RING16_W8_KB
#define G355_RING16_W8_KB 48
#endif
// The 256 x 256 tile holds one workgroup per CU (128 x 64 accumulators per
// wave): its ring may take most of the LDS.
#ifndef G355_RING16_BIG_KB
#define G355_RING16_BIG_KB 128
#endif
// The 16-bit 128 x 128 tile with the K-tile split between wave pairs holds
// one workgroup per CU: its ring takes most of the LDS.
#ifndef G355_RING16_K2_KB
#define G355_RING16_K2_KB 128
#endif

// Wait until at most n K-tiles of DPW transfers each are still in flight
// (0 <= n <= MAXT; n is the same on every lane).
template <int DPW, int MAXT> __device__ __forceinline__ void wait_tiles(int n) {
  [&]<int... t>(std::integer_sequence<int, t...>) {
    ((void)(n == t ? (wait_vm_lgkm0<t * DPW>(), 0) : 0), ...);
  }(std::make_integer_sequence<int, MAXT + 1>{});
}

template <int P, class S, bool TA, bool TB> struct DmaPlan {
  using T = Traits<P>;
  using E = typename T::E;
  // MN-contiguous operands of the one-element-per-lane MFMAs (binary64,
  // binary32): IL neighbouring 16-wide blocks take interleaved rows/columns
  // (block g*IL + t, lane c: index 16*IL*g + IL*c + t), so that a lane's
  // values for the IL blocks at one k are adjacent in LDS and come in one
  // read (ds_read_b128 for IL * element size = 16) instead of IL. The
  // epilogue maps the blocks back; every output element still receives the
  // same MFMA sequence.
  static constexpr int ES = (int)sizeof(E), VE = 16 / ES;
  static constexpr int ILA =
      (TA && T::KPL == 1 && ES >= 4) ? (VE < Geom<P, S>::FM ? VE : Geom<P, S>::FM) : 1;
  static constexpr int ILB =
      (!TB && T::KPL == 1 && ES >= 4) ? (VE < Geom<P, S>::FN ? VE : Geom<P, S>::FN) : 1;
  // Loader waves: every wave issues an equal share of a K-tile's 1 KiB
  // transfers; when the share is not whole (small tiles on 8 waves: a
  // 32 x 32 binary64 K-tile is 4 + 4 transfers), the first half or quarter
  // of the waves issue them, instead of the shape leaving the direct-to-LDS
  // path (32x32k2 at N = 2000: binary64 38.9 -> 47.2, binary32 51.6 -> 90.4
  // TFLOP/s). Where the share is whole, all waves issue: restricting the
  // 8-wave 128 x 128 binary64 tile to four loaders measured 4% slower.
  static constexpr int NW = S::NT / 64, BKD = bk_of<P, S>();
  static constexpr int TR_A = S::BM * BKD * ES / 1024, TR_B = S::BN * BKD * ES / 1024;
  static constexpr bool whole(int w) { return w >= 1 && TR_A % w == 0 && TR_B % w == 0; }
  static constexpr int LW = S::LDW > 0 ? S::LDW
                            : whole(NW) ? NW : whole(NW / 2) ? NW / 2 : whole(NW / 4) ? NW / 4 : NW;
  static constexpr int LT = 64 * LW;
  using OA = DmaOp<E, S::BM, BKD, LT, !TA, Geom<P, S>::KG, Geom<P, S>::MB, ILA * ES == 16>;
  using OB = DmaOp<E, S::BN, BKD, LT, TB, Geom<P, S>::KG, Geom<P, S>::MB, ILB * ES == 16>;
  static constexpr int STAGE = T::PLANES * (OA::BYTES + OB::BYTES);
  static constexpr int PER_WAVE = T::PLANES * (OA::PERW + OB::PERW);   // transfers per tile
  // Ring depth: transfers run NS - 1 K-tiles ahead of the MFMAs. binary64
  // and binary32: three stages when they fit in the ring budget, else two;
  // the budget is 72 KiB for 4-wave shapes, so that two workgroups share a
  // CU and one's barrier waits overlap the other's MFMAs (binary64 128 x 128
  // at N = 4096: 67.4 against 60.1 TFLOP/s with three stages and one
  // workgroup), and 144 KiB of the 160 KiB LDS for 8-wave shapes. 16-bit: as
  // many stages as fit in the 16-bit ring budget (2 to 8). vmcnt (6 bits)
  // bounds the transfers a wave may leave outstanding.
  static constexpr int R16 = S::KS > 1 ? G355_RING16_K2_KB * 1024
                             : (S::NT >= 512 && S::BM * S::BN <= 128 * 128) ? G355_RING16_W8_KB * 1024
                             : S::BM * S::BN >= 256 * 256 ? G355_RING16_BIG_KB * 1024
                                                          : kRing16;
  static constexpr int FIT = (T::KPL == 8 ? R16 : (S::NT <= 256 ? 72 : 144) * 1024) / STAGE;
  static constexpr int VMAX = 1 + 63 / (PER_WAVE > 0 ? PER_WAVE : 1);
  static constexpr int NS0 = T::KPL == 8 ? (FIT < 8 ? FIT : 8) : (FIT >= 3 ? 3 : 2);
  static constexpr int NS1 = NS0 < VMAX ? NS0 : VMAX;
  static constexpr int NS = NS1 < 2 ? 2 : NS1;
  static constexpr bool OK = OA::OK && OB::OK && Geom<P, S>::OK && PER_WAVE < 32 &&
                             NS * STAGE <= 160 * 1024 && (S::LDW == 0 || whole(S::LDW));
};

template <int P, class S, bool TA, bool TB> __host__ __device__ constexpr bool dma_ok() {
  return DmaPlan<P, S, TA, TB>::OK;
}

template <int P, class S, bool TA, bool TB> __host__ __device__ constexpr int lds_bytes_dma() {
  using T = Traits<P>;
  constexpr int stages = DmaPlan<P, S, TA, TB>::NS * DmaPlan<P, S, TA, TB>::STAGE;
  constexpr int red = S::KS > 1 ? S::BM * S::WTN * (int)sizeof(typename T::Acc) / 4 : 0;
  return stages > red ? stages : red;
}

// split_x for two elements at once: each term is one packed round-to-
// nearest-even conversion of the pair (v_cvt_pk_bf16_f32, the instruction
// the scalar conversion uses too), widened back to binary32 by a shift or a
// mask and subtracted exactly. o[p] holds term p of x0 in its low and of x1
// in its high 16 bits.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <int NP>
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t (&o)[NP]) {
  float r0 = x0, r1 = x1;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const f32x2 r = {r0, r1};
    const uint32_t w = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
    o[p] = w;
    if (p + 1 < NP) {
      r0 = r0 - __builtin_bit_cast(float, w << 16);
      r1 = r1 - __builtin_bit_cast(float, w & 0xffff0000u);
    }
  }
}

// Compute one BM x BN tile of C at (m0, n0) with direct-to-LDS operands.
// Same contract as gemm_tile with VEC = true.
template <int P, class S, bool TA, bool TB>
__device__ __forceinline__ void gemm_tile_dma(const GemmArgs &g, int64_t m0, int64_t n0,
                                              char *smem) {
  using T = Traits<P>;
  using GM = Geom<P, S>;
  using E = typename T::E;
  using Op = typename T::Op;
  using Acc = typename GM::Acc;
  using Out = typename T::Out;
  using Plan = DmaPlan<P, S, TA, TB>;
  using OA = typename Plan::OA;
  using OB = typename Plan::OB;
  static_assert(Plan::OK, "shape/layout not offered on the direct-to-LDS path");
  constexpr int BK = bk_of<P, S>(), KPL = T::KPL, PL = T::PLANES, KS = S::KS;
  constexpr int MB = GM::MB, FM = GM::FM, FN = GM::FN, NR = GM::NR;
  constexpr int KG = GM::KG, KW = KG / KS;
  constexpr int VE = 16 / (int)sizeof(E);
  constexpr int RU0 = VE < KW ? VE : KW;
  constexpr int RU = RU0 < KPL ? KPL : RU0;     // at least one MFMA operand
  constexpr int U = KW / RU, SPU = RU / KPL;
  constexpr int CV = T::CVT;
  constexpr int ILA = Plan::ILA, ILB = Plan::ILB;   // interleaved MN blocks (DmaPlan)
  static_assert(FM % ILA == 0 && FN % ILB == 0 && (ILA == 1 || MB == 16) && (ILB == 1 || MB == 16),
                "interleave");
  constexpr int NB = FM * FN, NB1 = NB / 2;
  constexpr int STAGE = Plan::STAGE, DPW = Plan::PER_WAVE;
  constexpr int NS = Plan::NS, D = NS - 1;     // ring stages, transfer distance in tiles

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform, in an SGPR
  const int wpos = wave % (S::WM * S::WN), kh = wave / (S::WM * S::WN);
  const int wm = wpos % S::WM, wn = wpos / S::WM;
  const int lr = lane % MB, lgp = lane / MB;

  // Waves that issue transfers: the loader waves of a shape that has them
  // (the others only compute), else all waves or the first LW of them.
  constexpr bool SPEC = S::LDW > 0;
  constexpr int CW = S::WM * S::WN * S::KS;     // compute waves
  const bool is_ld = SPEC && wave >= CW;
  const int lwave = SPEC ? (is_ld ? wave - CW : 0) : wave;   // index among the loaders
  const bool loader = SPEC ? is_ld : (Plan::LW == S::NT / 64 || wave < Plan::LW);
  const E *Ap[3] = {reinterpret_cast<const E *>(g.A), reinterpret_cast<const E *>(g.A2),
                    reinterpret_cast<const E *>(g.A3)};
  const E *Bp[3] = {reinterpret_cast<const E *>(g.B), reinterpret_cast<const E *>(g.B2),
                    reinterpret_cast<const E *>(g.B3)};
  OA oa;
  OB ob;
  oa.init(g.lda, m0, g.M, lwave, lane);
  ob.init(g.ldb, n0, g.N, lwave, lane);

  // region of plane pl of operand A / B in stage st
  auto regA = [&](int st, int pl) { return smem + st * STAGE + pl * OA::BYTES; };
  auto regB = [&](int st, int pl) { return smem + st * STAGE + PL * OA::BYTES + pl * OB::BYTES; };

  const int64_t KT = (g.K + BK - 1) / BK;
  auto issue_tile = [&](int64_t kt, int st) {
    if (!loader) return;
    const int64_t k0 = kt * BK;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) {
      const E *ta = TA ? Ap[pl] + k0 * g.lda + m0 : Ap[pl] + m0 * g.lda + k0;
      const E *tb = TB ? Bp[pl] + n0 * g.ldb + k0 : Bp[pl] + k0 * g.ldb + n0;
      oa.issue(ta, k0, g.K, regA(st, pl), lwave);
      ob.issue(tb, k0, g.K, regB(st, pl), lwave);
    }
  };

  Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = Acc{};

  using Unit = VecT<E, RU>;
  Unit fa[2][PL][FM], fb[2][PL][FN];
  auto read_unit = [&](int st, int u, auto buf_tag) {
    constexpr int b = decltype(buf_tag)::value;
    const int koff = lgp * KG + kh * KW + u * RU;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) {
      if constexpr (ILA > 1) {
#pragma unroll
        for (int gi = 0; gi < FM / ILA; ++gi)
#pragma unroll
          for (int e = 0; e < RU; ++e) {
            const auto v = OA::template read_row<ILA>(
                regA(st, pl), wm * S::WTM + gi * MB * ILA + ILA * lr, koff + e);
#pragma unroll
            for (int t = 0; t < ILA; ++t) fa[b][pl][gi * ILA + t].e[e] = v.e[t];
          }
      } else {
#pragma unroll
        for (int i = 0; i < FM; ++i)
          fa[b][pl][i] = OA::template read<RU>(regA(st, pl), wm * S::WTM + i * MB + lr, koff);
      }
      if constexpr (ILB > 1) {
#pragma unroll
        for (int gi = 0; gi < FN / ILB; ++gi)
#pragma unroll
          for (int e = 0; e < RU; ++e) {
            const auto v = OB::template read_row<ILB>(
                regB(st, pl), wn * S::WTN + gi * MB * ILB + ILB * lr, koff + e);
#pragma unroll
            for (int t = 0; t < ILB; ++t) fb[b][pl][gi * ILB + t].e[e] = v.e[t];
          }
      } else {
#pragma unroll
        for (int j = 0; j < FN; ++j)
          fb[b][pl][j] = OB::template read<RU>(regB(st, pl), wn * S::WTN + j * MB + lr, koff);
      }
    }
  };
  auto op_of = [](const auto &u, int step) {
    return *reinterpret_cast<const Op *>(&u.e[step * KPL]);
  };
  // In-register split (CV > 0): the bfloat16 terms of the current unit's
  // binary32 fragments, made right before the unit's MFMAs, two elements at
  // a time (bfloat16 pairs packed in 32 bits).
  using Half = VecT<uint32_t, (RU / 2 > 0 ? RU / 2 : 1)>;
  Half ca[CV > 0 ? CV : 1][FM], cb[CV > 0 ? CV : 1][FN];
  auto op_h = [](const Half &u, int step) {
    return *reinterpret_cast<const Op *>(&u.e[step * KPL / 2]);
  };
  auto convert = [&](auto buf_tag) {
    constexpr int b = decltype(buf_tag)::value;
    if constexpr (CV > 0) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int q = 0; q < RU / 2; ++q) {
          uint32_t t[CV];
          split_pair<CV>((float)fa[b][0][i].e[2 * q], (float)fa[b][0][i].e[2 * q + 1], t);
#pragma unroll
          for (int p = 0; p < CV; ++p) ca[p][i].e[q] = t[p];
        }
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int q = 0; q < RU / 2; ++q) {
          uint32_t t[CV];
          split_pair<CV>((float)fb[b][0][j].e[2 * q], (float)fb[b][0][j].e[2 * q + 1], t);
#pragma unroll
          for (int p = 0; p < CV; ++p) cb[p][j].e[q] = t[p];
        }
    }
  };

  // Issue of the transfers of the K-tile D ahead. binary64/binary32: spread
  // over the first half of the MFMAs issued before the barrier (a 1 KiB
  // transfer occupies the CU's address unit for many cycles, and a wave
  // queued behind it issues no MFMA meanwhile; transfer k goes right before
  // pre-barrier MFMA number k * NPRE / (2 DPW)), so the last one still has
  // half a K-tile to land before the barrier (spreading over the whole tile
  // measured 4-5% slower). 16-bit: all at the start of the K-tile, whose
  // MFMAs take about as long as the transfers themselves at the L2 -> CU
  // rate (measured 8-10% faster than spreading). A wave that issues no MFMA
  // before the barrier (one unit per K-tile and one block: the 8-wave
  // 32 x 32 tiles) has no slot to spread over and issues in one burst too.
  using TM = Terms<(CV > 0 ? CV : PL)>;
  constexpr int MPB = SPU * TM::N;                      // MFMAs per block per unit
  constexpr int NPRE = MPB * ((U - 1) * NB + NB1);       // pre-barrier MFMAs per tile
  constexpr bool BURST = KPL == 8 || NPRE == 0;
  struct Pending { srd_t sa[PL], sb[PL]; uint32_t la[PL], lb[PL]; int64_t k0; int32_t krem; bool on; };
  Pending pend;
  auto prep_tile = [&](int64_t kt, int st) {
    pend.on = kt < KT;
    if (!pend.on) return;
    {
      const int64_t rem = g.K - kt * BK;
      pend.krem = rem > 0x7fffffff ? 0x7fffffff : (int32_t)rem;
    }
    pend.k0 = kt * BK;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) {
      const E *ta = TA ? Ap[pl] + pend.k0 * g.lda + m0 : Ap[pl] + m0 * g.lda + pend.k0;
      const E *tb = TB ? Bp[pl] + n0 * g.ldb + pend.k0 : Bp[pl] + pend.k0 * g.ldb + n0;
      pend.sa[pl] = make_srd(ta);
      pend.sb[pl] = make_srd(tb);
      pend.la[pl] = lds_addr(regA(st, pl));
      pend.lb[pl] = lds_addr(regB(st, pl));
    }
  };
  auto issue_k = [&](auto k_tag) {   // transfer k of the pending tile
    constexpr int k = decltype(k_tag)::value;
    constexpr int per_plane = OA::PERW + OB::PERW;
    constexpr int pl = k / per_plane, r = k % per_plane;
    if (pend.on && loader) {
      if constexpr (r < OA::PERW)
        oa.issue_one(r, pend.sa[pl], pend.krem, pend.la[pl], lwave);
      else
        ob.issue_one(r - OA::PERW, pend.sb[pl], pend.krem, pend.lb[pl], lwave);
    }
  };
  // pre-barrier MFMA number n: issue every transfer k with k * NPRE / (2 DPW) == n
  auto maybe_issue = [&](auto n_tag) {
    constexpr int n = decltype(n_tag)::value;
    if constexpr (BURST || SPEC) return;
    [&]<int... k>(std::integer_sequence<int, k...>) {
      ((void)((k * NPRE / (2 * DPW) == n) ? (issue_k(std::integral_constant<int, k>{}), 0) : 0), ...);
    }(std::make_integer_sequence<int, DPW>{});
  };
  // MFMAs of blocks [lo, hi) of a unit; SLOT is the pre-barrier number of the
  // first one (or -1 after the barrier: no transfers there).
  auto mma_unit_s = [&](auto buf_tag, auto lo_tag, auto hi_tag, auto slot_tag) {
    constexpr int b = decltype(buf_tag)::value;
    constexpr int lo = decltype(lo_tag)::value, hi = decltype(hi_tag)::value;
    constexpr int SLOT = decltype(slot_tag)::value;
    constexpr int NX = hi - lo;
    if constexpr (CV > 0 && lo == 0) convert(buf_tag);
    [&]<int... m>(std::integer_sequence<int, m...>) {
      (([&] {
         constexpr int st = m / (TM::N * NX);
         constexpr int term = (m / NX) % TM::N;   // Terms order, smallest first
         constexpr int x = lo + m % NX;
         if constexpr (SLOT >= 0) maybe_issue(std::integral_constant<int, SLOT + m>{});
         if constexpr (CV > 0)
           mfma(acc[x / FN][x % FN], op_h(ca[TM::a[term]][x / FN], st),
                op_h(cb[TM::b[term]][x % FN], st));
         else
           mfma(acc[x / FN][x % FN], op_of(fa[b][TM::a[term]][x / FN], st),
                op_of(fb[b][TM::b[term]][x % FN], st));
       }()), ...);
    }(std::make_integer_sequence<int, SPU * TM::N * NX>{});
  };
  using I0 = std::integral_constant<int, 0>;
  using INB1 = std::integral_constant<int, NB1>;
  using INB = std::integral_constant<int, NB>;

  // One K-tile (stage cur): issue the transfers D tiles ahead (into the
  // stage read one tile ago), MFMAs on this tile, retire the next tile's
  // transfers, barrier, first fragments of the next tile under the last
  // half of this tile's MFMAs.
  auto ktile = [&](auto p0_tag, int64_t kt, int cur) {
    constexpr int P0 = decltype(p0_tag)::value;
    const int nxt = cur + 1 == NS ? 0 : cur + 1;
    if constexpr (!SPEC) prep_tile(kt + D, cur == 0 ? NS - 1 : cur - 1);
    if constexpr (BURST && !SPEC) {
      [&]<int... k>(std::integer_sequence<int, k...>) {
        (issue_k(std::integral_constant<int, k>{}), ...);
      }(std::make_integer_sequence<int, DPW>{});
    }
    [&]<int... u>(std::integer_sequence<int, u...>) {
      ((read_unit(cur, u + 1, std::integral_constant<int, (P0 + u + 1) & 1>{}),
        mma_unit_s(std::integral_constant<int, (P0 + u) & 1>{}, I0{}, INB{},
                   std::integral_constant<int, u * MPB * NB>{})), ...);
    }(std::make_integer_sequence<int, U - 1>{});
    constexpr int PLU = (P0 + U - 1) & 1;
    mma_unit_s(std::integral_constant<int, PLU>{}, I0{}, INB1{},
               std::integral_constant<int, (U - 1) * MPB * NB>{});
    if (kt + 1 < KT) {
      // tiles kt+2 .. min(kt+D, KT-1) may stay in flight
      const int64_t rest = KT - 2 - kt;
      wait_tiles<DPW, D - 1>(rest < D - 1 ? (int)rest : D - 1);
      raw_barrier();
      read_unit(nxt, 0, std::integral_constant<int, (P0 + U) & 1>{});
    }
    mma_unit_s(std::integral_constant<int, PLU>{}, INB1{}, INB{}, std::integral_constant<int, -1>{});
  };

  // Loader split (LCV planes): loader waves read the binary32 operands into
  // registers, two K-tiles ahead in two register sets, split every element
  // into LCV bfloat16 terms (split_pair, the rounding of the split step) and
  // write each term into its plane of the LDS stage, at the places the
  // plane transfers would fill. A chunk is one 16-byte LDS chunk of 8
  // elements: 32 bytes of binary32, read as two 16-byte halves; a half
  // outside the matrix reads as zeros (offset past the buffer record).
  constexpr int LCV = lcv_of<P>();
  static_assert(LCV == 0 || (SPEC && !TA && !TB && LCV == PL && KS == 2),
                "the loader split runs on loader-wave shapes, NN operands");
  constexpr int NCA = LCV ? OA::PERW : 0, NCB = LCV ? OB::PERW : 0, NCH = NCA + NCB;
  // per chunk: the byte offset of its binary32 data in the tile (rows of A,
  // K rows of B) and, packed, the K index the K edge is tested on (bits
  // 0-15) and which halves lie inside the M/N extent (bits 16-17); the LDS
  // place of chunk j is lds0 + j * 1 KiB * loader count
  uint32_t lvoff[NCH > 0 ? NCH : 1], lkm[NCH > 0 ? NCH : 1];
  const uint32_t lds0 = (uint32_t)(lwave * 1024 + lane * 16);
  u32x4 lbuf[2][NCH > 0 ? NCH : 1][2];
  auto lcv_setup = [&] {
    if constexpr (LCV > 0) {
#pragma unroll
      for (int j = 0; j < NCA; ++j) {     // A: row r, K offset k (K-contiguous)
        const int q = (lwave + j * OA::NW) * 64 + lane;
        const int r = q / OA::CPR, c = q % OA::CPR;
        const int k = (c ^ OA::swz(r)) * VE;
        lvoff[j] = (uint32_t)((r * g.lda + k) * 4);
        lkm[j] = (uint32_t)k | (m0 + r < g.M ? 3u << 16 : 0u);
      }
#pragma unroll
      for (int j = 0; j < NCB; ++j) {     // B: K row r, column m (N-contiguous)
        const int q = (lwave + j * OB::NW) * 64 + lane;
        const int r = q / OB::CPR, c = q % OB::CPR;
        const int mcol = (c ^ OB::swzm(r)) * VE;
        lvoff[NCA + j] = (uint32_t)((r * g.ldb + mcol) * 4);
        lkm[NCA + j] = (uint32_t)r | (n0 + mcol < g.N ? 1u << 16 : 0u) |
                       (n0 + mcol + 4 < g.N ? 2u << 16 : 0u);
      }
    }
  };
  auto lcv_load = [&](auto set_tag, int64_t kt) {
    constexpr int sx = decltype(set_tag)::value;
    const int64_t k0 = kt * BK;
    const int64_t rem = g.K - k0;
    const int32_t krem = rem > 0x7fffffff ? 0x7fffffff : (int32_t)rem;
    const __amdgpu_buffer_rsrc_t ra =
        make_rsrc(reinterpret_cast<const float *>(g.A) + m0 * g.lda + k0);
    const __amdgpu_buffer_rsrc_t rb =
        make_rsrc(reinterpret_cast<const float *>(g.B) + k0 * g.ldb + n0);
#pragma unroll
    for (int j = 0; j < NCH; ++j)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int32_t kidx = (int32_t)(lkm[j] & 0xffffu) + (j < NCA ? 4 * h : 0);
        const bool ok = ((lkm[j] >> (16 + h)) & 1u) && kidx < krem;
        lbuf[sx][j][h] = raw_load<16>(j < NCA ? ra : rb, ok ? lvoff[j] + 16u * h : kOob);
      }
  };
  auto lcv_store = [&](auto set_tag, int st) {
    constexpr int sx = decltype(set_tag)::value;
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      u32x4 o[LCV > 0 ? LCV : 1];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // elements taken out of the vector by value first: a bit cast of a
        // vector element in place read element 0 whatever the index
        const uint32_t u0 = lbuf[sx][j][e / 2][(e % 2) * 2];
        const uint32_t u1 = lbuf[sx][j][e / 2][(e % 2) * 2 + 1];
        uint32_t t[LCV > 0 ? LCV : 1];
        split_pair<(LCV > 0 ? LCV : 1)>(__builtin_bit_cast(float, u0),
                                        __builtin_bit_cast(float, u1), t);
#pragma unroll
        for (int p = 0; p < LCV; ++p) o[p][e] = t[p];
      }
#pragma unroll
      for (int p = 0; p < LCV; ++p) {
        const int slot = j < NCA ? j * OA::NW : (j - NCA) * OB::NW;
        char *dst = (j < NCA ? regA(st, p) : regB(st, p)) + lds0 + slot * 1024;
        *reinterpret_cast<u32x4 *>(dst) = o[p];
      }
    }
  };

  if (KT > 0) {
    if constexpr (LCV == 0) {
#pragma unroll
      for (int t = 0; t < D; ++t)
        if (t < KT) issue_tile(t, t);
      wait_tiles<DPW, D - 1>(KT < D ? (int)KT - 1 : D - 1);   // tile 0 has landed
    }
    static_assert(LCV == 0 || NS == 2, "loader split: two LDS stages");
    if constexpr (LCV == 0) raw_barrier();
    auto compute_loop = [&] {
      read_unit(0, 0, I0{});
      int st = 0;
      if constexpr (U % 2 == 0) {
        for (int64_t kt = 0; kt < KT; ++kt) {
          ktile(I0{}, kt, st);
          st = st + 1 == NS ? 0 : st + 1;
        }
      } else {
        for (int64_t kt = 0; kt < KT; kt += 2) {
          ktile(I0{}, kt, st);
          st = st + 1 == NS ? 0 : st + 1;
          if (kt + 1 < KT) {
            ktile(std::integral_constant<int, 1>{}, kt + 1, st);
            st = st + 1 == NS ? 0 : st + 1;
          }
        }
      }
    };
    if constexpr (LCV > 0) {
      // every use of the loaders' registers sits in this branch (the first
      // barrier too, duplicated in the compute branch), so that they share
      // no live range with the compute waves' registers
      if (is_ld) {
        lcv_setup();
        using I1 = std::integral_constant<int, 1>;
        // Loads of tiles past the end are issued too (every offset then lies
        // past the buffer record: zeros, no memory access), so that every
        // path carries the same loads in the same order and the compiler's
        // waits retire exactly the older register set, never the newer one.
        lcv_load(I0{}, 0);
        lcv_load(I1{}, 1);
        lcv_store(I0{}, 0);
        lcv_load(I0{}, 2);
        wait_vm_lgkm0<63>();     // the planes of tile 0 are written
        raw_barrier();
        // tile t is split into stage t % 2 from register set t % 2 once the
        // compute waves have passed the barrier that ends tile t - 2; then the
        // set takes tile t + 2
        for (int64_t kt = 0; kt < KT; kt += 2) {
          if (kt + 1 < KT) {
            lcv_store(I1{}, 1);
            lcv_load(I1{}, kt + 3);
            wait_vm_lgkm0<63>();
            raw_barrier();
          }
          if (kt + 2 < KT) {
            lcv_store(I0{}, 0);
            lcv_load(I0{}, kt + 4);
            wait_vm_lgkm0<63>();
            raw_barrier();
          }
        }
      } else {
        raw_barrier();
        compute_loop();
      }
    } else if constexpr (SPEC) {
      if (is_ld) {
        // loader waves: per K-tile, the transfers of the tile D ahead into
        // the stage read one tile ago, then the same waits and barriers as
        // the compute waves (which no longer wait on transfers of their own)
        int st = 0;
        for (int64_t kt = 0; kt < KT; ++kt) {
          prep_tile(kt + D, st == 0 ? NS - 1 : st - 1);
          [&]<int... k>(std::integer_sequence<int, k...>) {
            (issue_k(std::integral_constant<int, k>{}), ...);
          }(std::make_integer_sequence<int, DPW>{});
          if (kt + 1 < KT) {
            const int64_t rest = KT - 2 - kt;
            wait_tiles<DPW, D - 1>(rest < D - 1 ? (int)rest : D - 1);
            raw_barrier();
          }
          st = st + 1 == NS ? 0 : st + 1;
        }
      } else {
        compute_loop();
      }
    } else {
      compute_loop();
    }
    // every wave has finished its LDS reads before the stages are reused
    wait_vm_lgkm0<0>();
    raw_barrier();
  }

  // K-split tiles: the KS partial sums of each output are added through LDS.
  // Two-way splits whose partial tiles fit in the ring's LDS at once: each
  // wave of a pair keeps half of its blocks (kh 0 the first FM / 2 block
  // rows, kh 1 the rest), hands the other half to its partner and stores
  // only its own half (one exchange; every output is kh 0's sum plus kh 1's,
  // added in either order with the same result). Otherwise one wave column
  // at a time into the kh = 0 waves.
  using AEt = std::remove_reference_t<decltype(acc[0][0][0])>;
  constexpr bool HALVES = KS == 2 && FM % 2 == 0 &&
                          S::WM * S::WN * FM * FN * NR * 64 * (int)sizeof(AEt) <=
                              lds_bytes_dma<P, S, TA, TB>();
  auto owned = [&](int i) { return !HALVES || ((i < FM / 2) == (kh == 0)); };
  if constexpr (HALVES) {
    AEt *red = reinterpret_cast<AEt *>(smem);
    if (kh < KS) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
        if (!owned(i))
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < NR; ++q)
              red[(((wpos * FM + i) * FN + j) * NR + q) * 64 + lane] = acc[i][j][q];
    }
    __syncthreads();
    if (kh < KS) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
        if (owned(i))
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < NR; ++q)
              acc[i][j][q] += red[(((wpos * FM + i) * FN + j) * NR + q) * 64 + lane];
    }
    // the exchange is read before a persistent caller's next tile refills LDS
    __syncthreads();
    if (kh >= KS) return;   // loader waves
  } else if constexpr (KS > 1) {
    using AE = AEt;
    AE *red = reinterpret_cast<AE *>(smem);
#pragma unroll 1
    for (int col = 0; col < S::WN; ++col) {
#pragma unroll 1
      for (int h = 1; h < KS; ++h) {
        if (wn == col && kh == h) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
              for (int q = 0; q < NR; ++q)
                red[(((wm * FM + i) * FN + j) * NR + q) * 64 + lane] = acc[i][j][q];
        }
        __syncthreads();
        if (wn == col && kh == 0) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
              for (int q = 0; q < NR; ++q)
                acc[i][j][q] += red[(((wm * FM + i) * FN + j) * NR + q) * 64 + lane];
        }
        __syncthreads();
      }
    }
    if (kh != 0) return;
  } else if constexpr (SPEC) {
    if (is_ld) return;
  }

  constexpr int GRP = T::GRP, LGN = GM::LGN;
  // The 16-bit MFMA precisions store C with non-temporal stores (measured
  // at N = 2000: bf16 +3%, the two-way split +1.5%); binary64 stores lost
  // 3% that way and binary32 was level, so they keep ordinary stores.
  constexpr bool NTS = T::KPL == 8;
  Out *C = reinterpret_cast<Out *>(g.C);
  // Interleaved MN blocks (ILB > 1) leave a lane holding ILB neighbouring
  // columns of one row: they go out as one 8- or 16-byte store where C
  // allows it (base and row pitch aligned to the store, all ILB columns
  // inside N), else element by element.
  constexpr int VB = ILB * (int)sizeof(Out);
  constexpr int VS = (VB == 8 || VB == 16) ? ILB : 1;
  typedef Out OutV __attribute__((ext_vector_type(VS)));
  const bool cvec = VS > 1 && ((reinterpret_cast<uintptr_t>(g.C) |
                                (uintptr_t)(g.ldc * (int64_t)sizeof(Out))) & (VB - 1)) == 0;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    if (!owned(i)) continue;
#pragma unroll
    for (int j = 0; j < FN; j += VS) {
      const int64_t col = n0 + wn * S::WTN + (j / ILB) * MB * ILB + ILB * lr + j % ILB;
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const int r = (q / GRP) * LGN * GRP + lgp * GRP + q % GRP;   // row within the block
        const int64_t row = m0 + wm * S::WTM + (i / ILA) * MB * ILA + ILA * r + i % ILA;
        if (row >= g.M) continue;
        if (VS > 1 && cvec && col + VS <= g.N) {
          OutV v;
#pragma unroll
          for (int t = 0; t < VS; ++t) v[t] = (Out)acc[i][j + t][q];
          *reinterpret_cast<OutV *>(&C[row * g.ldc + col]) = v;
        } else {
#pragma unroll
          for (int t = 0; t < VS; ++t) {
            if (col + t < g.N) {
              if constexpr (NTS)
                __builtin_nontemporal_store((Out)acc[i][j + t][q], &C[row * g.ldc + col + t]);
              else
                C[row * g.ldc + col + t] = (Out)acc[i][j + t][q];
            }
          }
        }
      }
    }
  }
}

}  // namespace g355
