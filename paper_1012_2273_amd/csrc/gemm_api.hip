// gemm_api.hip -- the C ABI: argument validation, tile-shape choice,
// dispatch, grouped plans (planner, autotuner, hipGraph capture).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <tuple>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "gemm_mi355x.h"
#include "gemm_mi355x_tuning.h"
#include "gemm_tile.hpp"
#include "internal.h"

namespace g355 {

static thread_local std::string t_err;

int set_error(int code, const std::string &detail) {
  t_err = detail;
  return code;
}
void clear_error() { t_err.clear(); }

static const CfgInfo kCfgs[CFG_COUNT] = {{128, 128, "128x128"}, {128, 64, "128x64"},
                                         {64, 64, "64x64"},     {32, 32, "32x32"},
                                         {128, 128, "128x128w8"}, {128, 128, "128x128k2"},
                                         {128, 64, "128x64k2"},   {64, 64, "64x64k2"},
                                         {32, 32, "32x32k2"},     {128, 256, "128x256w8"},
                                         {64, 64, "64x64k4"},     {128, 128, "128x128k2ld"},
                                         {256, 256, "256x256w8"}};
const CfgInfo &cfg_info(int id) { return kCfgs[id]; }

// Tuning knobs (gemm_mi355x_tuning.h): per calling thread, so a test or a
// tuning tool that forces a shape never changes another thread's launches.
static thread_local int t_force_cfg = -1;
static thread_local int t_force_parts = -1;
// Forms of the split products (split_form below); -1 lets the sizes decide.
enum SplitForm : int { FORM_TWO_STEP = 0, FORM_REGISTERS = 1, FORM_LOADERS = 2 };
static thread_local int t_force_form = -1;

// The K-split shapes divide a 16-deep K-tile between two waves; the 16-bit
// paths take 32-deep K-tiles of 8-element MFMA steps and do not offer them.
// The 128x256w8 shape is offered to the bfloat16-MFMA products only.
bool cfg_supported(int prec, int cfg) {
  if (cfg < 0 || cfg >= CFG_COUNT) return false;
  if (cfg == CFG_128x128_K2 || cfg == CFG_128x128_K2_LD)   // 16-bit, loaders: direct-to-LDS only
    return true;
  if (cfg == CFG_128x128_W8) return true;   // also a grouped shape
  if (cfg_grouped(cfg)) return prec == PREC_F64 || prec == PREC_F32;
  if (cfg == CFG_128x256_W8) return prec != PREC_F64 && prec != PREC_F32;
  if (cfg == CFG_256x256_W8) return prec == PREC_BF16 || prec == PREC_SPLIT || prec == PREC_FSPLIT;
  if (cfg == CFG_64x64_K4) return prec == PREC_F64;
  return true;
}
bool cfg_grouped(int cfg) {
  for (int c : kGroupedCfgs)
    if (c == cfg) return true;
  return false;
}

static int device_cus() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  cache[dev] = cus;
  return cus;
}

// Tile shape for one product, from measured sweeps on MI355X (square
// products N = 500 .. 8192, every shape forced in turn). The deciding
// quantity is the number t of 128 x 128 tiles of C against the 256 CUs:
//  * fewer than ~48: small tiles occupy the CUs;
//  * up to ~200: medium shapes. binary64: one 16-wave 64 x 64 workgroup per
//    CU with K split four ways up to ~80 (N = 1000: 41.8 against 37.5
//    TFLOP/s for the 4-wave tile, N = 800: 27.1 against 24.4), 32 x 32 up
//    to ~110 (below), 64 x 64 above;
//  * up to one tile per CU: one 8-wave workgroup per CU (binary64: 4 x 2
//    waves of 32 x 64, 1.5% ahead of the K split at N = 1800 .. 3000;
//    binary32: 128 x 64 K split; 16-bit: 128 x 128 with 8 waves);
//  * more: binary64/binary32 the 4-wave 128 x 128 tile, two workgroups per
//    CU (binary64 ~2% ahead of the 8-wave tile at N = 2500 and 2800,
//    binary32 91.6 -> 98.6 and 115.6 -> 123.9 TFLOP/s against the 128 x 64
//    K split there); 16-bit from two tiles per CU the 128 x 256 tile, which
//    moves fewer operand bytes per flop.
static int choose_rule(int prec, int64_t m, int64_t n) {
  const int64_t t128 = ((m + 127) / 128) * ((n + 127) / 128);
  const int64_t cus = device_cus();
  const int64_t big = cus * 200 / 256, mid = cus * 48 / 256;
  switch (prec) {
    case PREC_F64:
      if (t128 > cus) return CFG_128x128;
      if (t128 >= big) return CFG_128x128_W8;
      if (t128 >= mid) {
        if (t128 <= cus * 80 / 256) return CFG_64x64_K4;
        // 324..361 tiles of 64 x 64 leave a fifth to two fifths of the CUs
        // with a second tile; 32 x 32 tiles spread evenly (N = 1100: 36.3
        // against 30.5 TFLOP/s, N = 1200: 38.3 against 36.5; 64 x 64 again
        // ahead from N = 1300, 41.9 against 37.4)
        return t128 <= cus * 110 / 256 ? CFG_32x32 : CFG_64x64;
      }
      return CFG_32x32;
    case PREC_F32:
      if (t128 > cus) return CFG_128x128;
      if (t128 >= big) return CFG_128x64_K2;
      return t128 >= mid ? CFG_64x64_K2 : CFG_32x32;
    // 16-bit, measured on MI355X with random operands (TFLOP/s, the tile the
    // rule takes against the best other): the 128 x 128 tile with loader
    // waves holds a CU by itself (its ring takes 128 KiB of LDS) and still
    // leads from about a quarter of a tile per CU up, also where its tiles
    // take a second, partial round -- bf16 N = 1200 196 against 149
    // (64 x 64), 2600 615 against 568 (the 8-wave tile, three of which share
    // a CU), 2800 721 against 608 -- and bf16 takes the 128 x 256 tile from
    // two tiles per CU (N = 3000 619 against 587, 4096 984 against 877). The
    // split planes keep the loader tile at every size measured (nominal
    // 2N^3/t: N = 1500 150 against 118, 3000 257 against 199, 4096 351
    // against 334, 5000 315 against 280, 8192 345 against 329). From two
    // tiles per CU both take the 256 x 256 tile, a third fewer operand bytes
    // per flop than 128 x 256 (bf16 N = 4096 1037 against 1000, 5000 900
    // against 821, 8192 1124 against 985, 6144 918 against 934; split N =
    // 3000 266 against 254, 4096 396 against 354, 5000 333 against 311, 6144
    // 314 against 304, 8192 385 against 346). Operands without 16-byte rows
    // have no loader or 256 x 256 tile: fallback_rule below.
    case PREC_BF16:
      if (t128 >= 2 * cus) return CFG_256x256_W8;
      return t128 >= mid ? CFG_128x128_K2_LD : CFG_32x32;
    case PREC_SPLIT:
      if (t128 >= 2 * cus) return CFG_256x256_W8;
      if (2 * t128 >= cus) return CFG_128x128_K2_LD;
      return t128 >= mid ? CFG_64x64 : CFG_32x32;
    // the two-way split in registers (small products, see split_form): the
    // loader tile from half a tile per CU (N = 1500 163 against 109)
    case PREC_FSPLIT:
      if (2 * t128 >= cus) return CFG_128x128_K2_LD;
      return t128 >= mid ? CFG_64x64 : CFG_32x32;
    default:  // three planes, three-way fused split
      if (t128 >= 2 * cus) return CFG_128x256_W8;
      if (t128 >= big) return CFG_128x128_W8;
      return t128 >= mid ? CFG_64x64 : CFG_32x32;
  }
}

// The 16-bit choice where the rule's tile is not offered (operands that
// need the register path: rows that are not 16-byte multiples): the 8-wave
// tile from about one tile per CU, three of whose workgroups share a CU.
static int fallback_rule(int prec, int64_t m, int64_t n) {
  const int64_t t128 = ((m + 127) / 128) * ((n + 127) / 128);
  const int64_t cus = device_cus();
  const int64_t big = cus * 200 / 256, mid = cus * 48 / 256;
  if ((prec == PREC_BF16 || prec == PREC_SPLIT) && t128 >= 2 * cus) return CFG_128x256_W8;
  if (t128 >= big) return CFG_128x128_W8;
  return t128 >= mid ? CFG_64x64 : CFG_32x32;
}

// Workgroups one CU holds for a kernel, cached per device.
static int occupancy(int prec, int layout, int cfg, int vw) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  const auto key = std::make_tuple(dev, prec, layout, cfg, vw);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int occ = plain_occupancy(prec, layout, cfg, vw);
  if (occ <= 0) occ = 1;
  cache[key] = occ;
  return occ;
}

// Large-N rate (TFLOP/s, square NN products N = 4096-8192 on MI355X) of the
// binary64/binary32 shapes the round-count check compares (binary64 128 x 64:
// about 0.93 of 128 x 128, its ratio at N = 6000).
static double shape_rate(int prec, int cfg) {
  if (prec == PREC_F64) {
    switch (cfg) {
      case CFG_128x128: return 69.2;
      case CFG_128x64: return 64.5;
      case CFG_128x128_W8: return 68.2;
      case CFG_128x128_K2: return 67.4;
      case CFG_64x64: return 62.2;
    }
  } else {
    switch (cfg) {
      case CFG_128x128: return 136.6;
      case CFG_128x64_K2: return 128.8;
      case CFG_64x64_K2: return 122.2;
    }
  }
  return 0.0;
}

// Time estimate of a shape in whole rounds of the device's workgroup slots:
// rounds x (tiles a CU holds per round x tile area) / large-N rate.
// Round counting: WHOLE counts every started round in full; FRACTION counts
// the last round by how full it is (freed slots take the next tiles as
// workgroups finish); ALONE counts a last round that gives each CU at most
// one workgroup as half a round (a workgroup alone on a CU runs about twice
// as fast as one sharing it).
enum RoundCount { WHOLE, FRACTION, ALONE };
static double round_cost(int prec, int layout, int vw, int cfg, int64_t m, int64_t n,
                         RoundCount mode = WHOLE) {
  const int bm = kCfgs[cfg].bm, bn = kCfgs[cfg].bn;
  const int64_t tiles = ((m + bm - 1) / bm) * ((n + bn - 1) / bn);
  const int occ = occupancy(prec, layout, cfg, vw);
  const int64_t cus = device_cus(), slots = cus * occ;
  const int64_t full = tiles / slots, last = tiles - full * slots;
  double rounds;
  if (mode == FRACTION) rounds = (double)tiles / slots;
  else if (mode == ALONE && last > 0 && last <= cus) rounds = full + 0.55;
  else rounds = (double)(full + (last > 0 ? 1 : 0));
  return rounds * occ * bm * bn / shape_rate(prec, cfg);
}

// The rule above ignores how full the last round of workgroups is: at
// N = 3000 binary64, 576 tiles of 128 x 128 take two rounds of 512 slots
// (46 TFLOP/s) where 2209 tiles of 64 x 64 fill three rounds of 768 (57).
// binary64/binary32 step down to the 64 x 64 shape when the round count
// says it is at least 15% faster.
static int choose_cfg(int prec, int layout, int vw, int64_t m, int64_t n) {
  const int forced = t_force_cfg;
  if (forced >= 0 && forced < CFG_COUNT && cfg_supported(prec, forced) &&
      plain_offered(prec, layout, forced, vw))
    return forced;
  int pick = choose_rule(prec, m, n);
  // shapes offered on the direct-to-LDS path only (loader waves, 16-bit K
  // split) step back where the operands need the register path or the
  // layout has no such kernel
  if (!plain_offered(prec, layout, pick, vw)) pick = fallback_rule(prec, m, n);
  if (!plain_offered(prec, layout, pick, vw)) pick = CFG_128x128_W8;
  // Plain products just above the small tier: while the 32 x 32 tiles fit
  // in one round of the workgroups the CUs hold, they beat the mid-tier
  // shapes (binary64 N = 800: 625 tiles in 768 slots, 31.0 against 35.9 us
  // on the 16-wave 64 x 64 tile; binary32 21.7 -> 18.6, bf16 11.5 -> 10.1;
  // N = 896: 784 tiles, a second round, 39.6 against 39.6, binary32 27.5
  // against 23.8)
  if ((prec == PREC_F64 || prec == PREC_F32 || prec == PREC_BF16) && pick != CFG_32x32 &&
      plain_offered(prec, layout, CFG_32x32, vw)) {
    const int64_t t32 = ((m + 31) / 32) * ((n + 31) / 32);
    if (t32 <= device_cus() * (int64_t)occupancy(prec, layout, CFG_32x32, vw)) pick = CFG_32x32;
  }
  if (prec != PREC_F64 && prec != PREC_F32) return pick;
  const int alt = prec == PREC_F64 ? CFG_64x64 : CFG_64x64_K2;
  if (kCfgs[pick].bm < 128 || shape_rate(prec, pick) <= 0.0) return pick;
  const double cp = round_cost(prec, layout, vw, pick, m, n);
  const double ca = round_cost(prec, layout, vw, alt, m, n);
  if (ca < 0.85 * cp) return alt;
  // The 64 x 64 shapes hold several workgroups per CU, so their last round
  // fills as slots free up: compare their fractional rounds too (N = 3600:
  // 3249 tiles of 64 x 64 over 768 slots against 841 of 128 x 128 over 512;
  // binary64 58.1 against 53.2 TFLOP/s, binary32 113.1 against 104.2), unless
  // whole rounds make them clearly slower (N = 2500: 3 rounds against 1, a 1%
  // loss). A last round of the large shape that leaves each CU at most one
  // workgroup runs at about twice the rate and counts as half a round
  // (N = 4300: 132 such tiles; binary64 59.8 with 128 x 128 against 56.3
  // with 64 x 64, binary32 117.9 against 110.7).
  const double cph = round_cost(prec, layout, vw, pick, m, n, ALONE);
  const double caf = round_cost(prec, layout, vw, alt, m, n, FRACTION);
  if (caf < 0.90 * cph && ca < 1.10 * cp) return alt;
  // A 128 x 128 pick is also weighed against the 128 x 64 shape (N = 4500:
  // 1296 tiles of 128 x 128 fill a third round of 512 slots only to 272;
  // 128 x 64 gives binary64 60.0 TFLOP/s against 55.1, its K split binary32
  // 122.5 against 108.9)
  const int mid = prec == PREC_F64 ? CFG_128x64 : CFG_128x64_K2;
  if (pick == CFG_128x128 && round_cost(prec, layout, vw, mid, m, n, ALONE) < 0.90 * cph)
    return mid;
  return pick;
}

static size_t esize_of(int dtype) {
  switch (dtype) {
    case GEMM_F64: return 8;
    case GEMM_F32: return 4;
    case GEMM_BF16: return 2;
  }
  return 0;
}

// Vector loads of `bytes` (16 or 8) need an aligned base and row pitch, and
// a contiguous extent that is a whole number of vectors (every vector is
// then entirely inside or outside the matrix).
static bool vec_ok(const void *p, int64_t ld, size_t es, int64_t contiguous_extent,
                   int bytes = 16) {
  const int64_t v = bytes / (int64_t)es;
  return v >= 1 && ((uintptr_t)p % bytes == 0) && (((uint64_t)ld * es) % bytes == 0) &&
         (contiguous_extent % v == 0);
}

// Operand offsets inside a tile are 32-bit and offsets from 2^31 on read as
// zeros: the largest tile (256 rows of the 128 x 256 shape) must span less
// than 2^31 bytes, so row pitches stay below 8 MiB.
constexpr uint64_t kMaxPitch = 1ull << 23;
static int check_ld_range(const char *name, int64_t ld, size_t es) {
  if ((uint64_t)ld * es >= kMaxPitch)
    return set_error(GEMM_EINVAL, std::string("leading dimension of ") + name +
                                      " too large (row pitch must be below 8 MiB)");
  return GEMM_OK;
}

static int hip_fail(hipError_t e, const char *what) {
  return set_error(GEMM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Shared validation for a row-major (rows x cols) operand.
static int check_mat(const char *name, const void *p, int64_t rows, int64_t cols, int64_t ld) {
  if (rows > 0 && cols > 0 && p == nullptr)
    return set_error(GEMM_ENULL, std::string(name) + " is NULL");
  if (ld < cols || ld < 0)
    return set_error(GEMM_ELD, std::string("leading dimension of ") + name + " (" +
                                   std::to_string(ld) + ") < row length " + std::to_string(cols));
  return GEMM_OK;
}

static int run_product(int prec, int layout, const GemmArgs &a, size_t es_in, hipStream_t s) {
  if (a.M == 0 || a.N == 0) return GEMM_OK;
  int rc;
  if ((rc = check_ld_range("A", a.lda, es_in)) || (rc = check_ld_range("B", a.ldb, es_in)))
    return rc;
  const bool ta = layout == LAYOUT_TN, tb = layout == LAYOUT_NT;
  const int64_t ea = ta ? a.M : a.K, eb = tb ? a.K : a.N;   // contiguous extents
  // widest vector loads both operands allow: 16 bytes (direct-to-LDS when the
  // shape offers it), 8 bytes (register path; 2- and 4-byte elements), else
  // single elements
  int vw = 0;
  if (vec_ok(a.A, a.lda, es_in, ea) && vec_ok(a.B, a.ldb, es_in, eb))
    vw = 16;
  else if (es_in < 8 && vec_ok(a.A, a.lda, es_in, ea, 8) && vec_ok(a.B, a.ldb, es_in, eb, 8))
    vw = 8;
  if (prec == PREC_SPLIT || prec == PREC_SPLIT3) vw = 16;   // planes are padded to whole vectors
  const int cfg = choose_cfg(prec, layout, vw, a.M, a.N);
  hipError_t e = launch_plain(prec, layout, cfg, vw, a, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return GEMM_OK;
}

static int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Widest vector loads both operands of an NN product allow.
static int nn_vector_width(const GemmArgs &a, size_t es) {
  if (vec_ok(a.A, a.lda, es, a.K) && vec_ok(a.B, a.ldb, es, a.N)) return 16;
  if (es < 8 && vec_ok(a.A, a.lda, es, a.K, 8) && vec_ok(a.B, a.ldb, es, a.N, 8)) return 8;
  return 0;
}

// K split over workgroups for products with too few output tiles to occupy
// the device: the tile shape, the number of K chunks and their length kc (a
// multiple of 64, so every chunk but the last holds whole K-tiles of every
// precision and starts 16-byte aligned). 64 x 64 tiles, chunks for about
// three workgroups per CU, each at least 128 deep; binary64 splits while its
// 64 x 64 tiles number at most two per CU, binary32 and bf16 (whose plain
// mid-size shapes already split K inside the workgroup) at most one per two
// CUs. binary64 products whose 128 x 128 tiles, one per CU, leave chunks
// at least 1024 deep take the 8-wave 128 x 128 shape instead (twice the
// flops per operand byte of 64 x 64). Measured on MI355X (TFLOP/s, binary64):
// N = 800 26.7 -> 30.7, N = 1200 36.3 -> 43.7, 256 x 256 x 65536 5.5 -> 59.0
// (64 chunks of 128 x 128; 52.3 with 47 of 64 x 64), 512 x 512 x 16384
// 21.5 -> 59.8, 1024 x 1024 x 8192 51.0 -> 64.0; binary32 N = 1000 would
// lose (67.2 -> 60.7) and stays unsplit. binary32 and bf16 products whose
// 128 x 128 tiles, two per CU, leave chunks at least 512 deep take that
// shape (1024 x 1024 x 8192: binary32 91.3 -> 117.0 against the 64 x 64
// rule, bf16 188.5 -> 455.7; 256 x 256 x 65536: binary32 10.2 unsplit, 79.7
// with 64 x 64, 92.1).
// Depends only on the precision, the sizes, the device and the forced
// settings, so the workspace query and the product agree.
struct KsplitPlan { int cfg, parts; int64_t kc; };
static KsplitPlan ksplit_plan(int prec, int64_t m, int64_t n, int64_t k) {
  KsplitPlan p{CFG_64x64, 1, k};
  const int fc = t_force_cfg;
  if (fc >= 0 && fc < CFG_COUNT && ksplit_offered(prec, LAYOUT_NN, fc, 16)) p.cfg = fc;
  const int bm = kCfgs[p.cfg].bm, bn = kCfgs[p.cfg].bn;
  const int64_t tiles = ((m + bm - 1) / bm) * ((n + bn - 1) / bn);
  const int64_t cus = device_cus();
  int64_t parts = 1;
  const int fp = t_force_parts;
  // binary64 with deep chunks: 128 x 128 tiles of 8 waves, one workgroup per
  // CU, when chunks of at least 1024 indices fill the device
  const int64_t t128 = ((m + 127) / 128) * ((n + 127) / 128);
  // binary32/bf16 likewise with 4-wave 128 x 128 tiles, two per CU, when
  // chunks of at least 512 indices fill the device
  if (fp <= 0 && fc < 0 && prec == PREC_F64 && t128 > 0 && 2 * t128 <= cus &&
      k / 1024 >= cus / t128) {
    p.cfg = CFG_128x128_W8;
    parts = cus / t128;
  } else if (fp <= 0 && fc < 0 && prec != PREC_F64 && t128 > 0 && t128 <= cus &&
             k / 512 >= 2 * cus / t128) {
    p.cfg = CFG_128x128;
    parts = 2 * cus / t128;
  } else if (fp > 0) {
    parts = fp;
  } else if (tiles > 0 && tiles <= (prec == PREC_F64 ? 2 * cus : cus / 2)) {
    const int64_t by_slots = 3 * cus / tiles, by_k = k / 128;
    parts = by_slots < by_k ? by_slots : by_k;
    if (parts > 1024) parts = 1024;
  }
  if (k <= 0 || parts <= 1) return p;
  p.kc = round_up((k + parts - 1) / parts, 64);
  p.parts = (int)((k + p.kc - 1) / p.kc);
  return p;
}

static size_t ksplit_bytes(int prec, const KsplitPlan &p, int64_t m, int64_t n) {
  return p.parts <= 1 ? 0 : (size_t)(p.parts - 1) * m * n * (prec == PREC_F64 ? 8 : 4);
}

// Scratch of the allocation-free K split (gemm_plain_ksplit_noalloc): the
// partial-product planes live in this array instead of a caller workspace.
// Each device holds its own copy from the library's load on that device to
// the end of the process. In host code `scratch` is only a handle for the
// symbol lookup; its device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address reaches kernels.
// Every chunk writes its whole plane before the sum reads it, so nothing in
// the array needs clearing between calls.
static __device__ __attribute__((aligned(256))) char scratch[GEMM_NOALLOC_SCRATCH_BYTES];

static void *scratch_device_address(int *rc) {
  static std::mutex mu;
  static std::map<int, void *> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *rc = hip_fail(e, "hipGetDevice");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    *rc = e != hipSuccess ? hip_fail(e, "hipGetSymbolAddress(scratch)")
                          : set_error(GEMM_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
    return nullptr;
  }
  addr[dev] = p;
  return p;
}

}  // namespace g355

using namespace g355;

extern "C" {

const char *gemm_strerror(int status) {
  switch (status) {
    case GEMM_OK: return "success";
    case GEMM_EINVAL: return "invalid argument";
    case GEMM_ENULL: return "null pointer";
    case GEMM_ELD: return "leading dimension too small";
    case GEMM_EWORKSPACE: return "workspace too small";
    case GEMM_EUNSUPPORTED: return "unsupported dtype";
    case GEMM_EHIP: return "HIP runtime error";
    case GEMM_ENOMEM: return "out of memory";
    case GEMM_ESTATE: return "invalid plan state";
  }
  return "unknown status";
}

const char *gemm_last_error(void) { return t_err.c_str(); }

int gemm_tile_config_count(void) { return CFG_COUNT; }

const char *gemm_tile_config_name(int id) {
  if (id < 0 || id >= CFG_COUNT) return "";
  return kCfgs[id].name;
}

int gemm_tuning_force_tile_config(int id) {
  clear_error();
  if (id >= CFG_COUNT || id < -1) return set_error(GEMM_EINVAL, "tile config id out of range");
  t_force_cfg = id;
  return GEMM_OK;
}

int gemm_plain(int dtype, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
               const void *B, int64_t ldb, void *C, int64_t ldc, void *stream) {
  clear_error();
  if (dtype != GEMM_F64 && dtype != GEMM_F32 && dtype != GEMM_BF16)
    return set_error(GEMM_EUNSUPPORTED, "dtype " + std::to_string(dtype));
  if (m < 0 || n < 0 || k < 0) return set_error(GEMM_EINVAL, "negative size");
  int rc;
  if ((rc = check_mat("A", A, m, k, lda)) || (rc = check_mat("B", B, k, n, ldb)) ||
      (rc = check_mat("C", C, m, n, ldc)))
    return rc;
  if (m == 0 || n == 0) return GEMM_OK;
  GemmArgs a{m, n, k, A, lda, B, ldb, nullptr, nullptr, C, ldc};
  const int prec = dtype == GEMM_F64 ? PREC_F64 : dtype == GEMM_F32 ? PREC_F32 : PREC_BF16;
  return run_product(prec, LAYOUT_NN, a, esize_of(dtype), (hipStream_t)stream);
}


// Workspace layout: the np planes of A (m rows each), then the np planes of
// B transposed (n rows each), hi first; each plane starts on a 256-byte
// boundary. Plane rows hold kp = k rounded up to 8 elements (zeros past k,
// so every plane row is a whole number of 16-byte vectors) at a pitch
// of ldp = kp rounded up to 64 elements: every row starts on a 128-byte
// line, so a 16-byte-per-lane transfer of a K-tile touches whole lines
// (a 4000-byte pitch at k = 2000 made most K-chunks straddle two lines and
// cost the product 17% at N = 2000).
static int plain_prec(int dtype) {
  return dtype == GEMM_F64 ? PREC_F64 : dtype == GEMM_F32 ? PREC_F32 : PREC_BF16;
}

int gemm_tuning_force_split_form(int form) {
  clear_error();
  if (form < -1 || form > FORM_LOADERS) return set_error(GEMM_EINVAL, "split form out of range");
  t_force_form = form;
  return GEMM_OK;
}

int gemm_tuning_force_ksplit_parts(int parts) {
  clear_error();
  if (parts < -1 || parts == 0 || parts > 65535)
    return set_error(GEMM_EINVAL, "K chunk count out of range");
  t_force_parts = parts;
  return GEMM_OK;
}

size_t gemm_plain_ksplit_workspace_size(int dtype, int64_t m, int64_t n, int64_t k) {
  if (dtype != GEMM_F64 && dtype != GEMM_F32 && dtype != GEMM_BF16) return 0;
  if (m <= 0 || n <= 0 || k <= 0) return 0;
  const int prec = plain_prec(dtype);
  return ksplit_bytes(prec, ksplit_plan(prec, m, n, k), m, n);
}

// Validation, plan and launches of the K split, shared by gemm_plain_ksplit
// (caller workspace) and gemm_plain_ksplit_noalloc (the per-device scratch
// array below): `ws` is a device address of at least `ws_bytes` bytes, or
// NULL when `ws_bytes` is 0.
static int ksplit_product(int dtype, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                          const void *B, int64_t ldb, void *C, int64_t ldc, void *(*get_ws)(int *),
                          void *workspace, size_t workspace_bytes, void *stream) {
  if (dtype != GEMM_F64 && dtype != GEMM_F32 && dtype != GEMM_BF16)
    return set_error(GEMM_EUNSUPPORTED, "dtype " + std::to_string(dtype));
  if (m < 0 || n < 0 || k < 0) return set_error(GEMM_EINVAL, "negative size");
  int rc;
  if ((rc = check_mat("A", A, m, k, lda)) || (rc = check_mat("B", B, k, n, ldb)) ||
      (rc = check_mat("C", C, m, n, ldc)))
    return rc;
  if (m == 0 || n == 0) return GEMM_OK;
  const int prec = plain_prec(dtype);
  const size_t es = esize_of(dtype);
  GemmArgs a{m, n, k, A, lda, B, ldb, nullptr, nullptr, C, ldc};
  hipStream_t s = (hipStream_t)stream;
  const KsplitPlan p = ksplit_plan(prec, m, n, k);
  if (p.parts <= 1) return run_product(prec, LAYOUT_NN, a, es, s);
  const size_t need = ksplit_bytes(prec, p, m, n);
  if (get_ws) {
    if (need > workspace_bytes)
      return set_error(GEMM_EWORKSPACE, "the K split of this product needs " +
                                            std::to_string(need) +
                                            " bytes of scratch; the allocation-free call holds " +
                                            std::to_string(workspace_bytes));
    if ((rc = check_ld_range("A", lda, es)) || (rc = check_ld_range("B", ldb, es))) return rc;
    if (!(workspace = get_ws(&rc))) return rc;
  } else {
    if (workspace == nullptr || workspace_bytes < need)
      return set_error(GEMM_EWORKSPACE, "need " + std::to_string(need) + " bytes, got " +
                                            std::to_string(workspace_bytes));
    if ((uintptr_t)workspace % 16 != 0)
      return set_error(GEMM_EWORKSPACE, "workspace must be 16-byte aligned");
    if ((rc = check_ld_range("A", lda, es)) || (rc = check_ld_range("B", ldb, es))) return rc;
  }
  const int vw = nn_vector_width(a, es);
  if (!ksplit_offered(prec, LAYOUT_NN, p.cfg, vw))
    return set_error(GEMM_EINVAL, "tile config not offered for the K split");
  hipError_t e = launch_ksplit(prec, LAYOUT_NN, p.cfg, vw, a, p.parts, p.kc, workspace, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  e = launch_ksplit_sum(prec, C, ldc, workspace, m, n, p.parts - 1, s);
  if (e != hipSuccess) return hip_fail(e, "sum launch");
  return GEMM_OK;
}

int gemm_plain_ksplit(int dtype, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                      const void *B, int64_t ldb, void *C, int64_t ldc, void *workspace,
                      size_t workspace_bytes, void *stream) {
  clear_error();
  return ksplit_product(dtype, m, n, k, A, lda, B, ldb, C, ldc, nullptr, workspace,
                        workspace_bytes, stream);
}

int gemm_plain_ksplit_noalloc(int dtype, int64_t m, int64_t n, int64_t k, const void *A,
                              int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc,
                              void *stream) {
  clear_error();
  return ksplit_product(dtype, m, n, k, A, lda, B, ldb, C, ldc, scratch_device_address, nullptr,
                        GEMM_NOALLOC_SCRATCH_BYTES, stream);
}

static void split_layout(int np, int64_t m, int64_t n, int64_t k, int64_t &kp, int64_t &ldp,
                         size_t off[6], size_t &total) {
  kp = round_up(k > 0 ? k : 1, 8);
  ldp = round_up(kp, 64);
  const size_t a_bytes = (size_t)round_up(m * ldp * 2, 256);
  const size_t b_bytes = (size_t)round_up(n * ldp * 2, 256);
  // A planes first, then B planes: off[p] = A plane p, off[np + p] = B plane p
  for (int p = 0; p < np; ++p) {
    off[p] = p * a_bytes;
    off[np + p] = np * a_bytes + p * b_bytes;
  }
  total = np * (a_bytes + b_bytes);
}

size_t gemm_split_workspace_size(int64_t m, int64_t n, int64_t k) {
  if (m < 0 || n < 0 || k < 0) return 0;
  int64_t kp, ldp;
  size_t off[6], total;
  split_layout(2, m, n, k, kp, ldp, off, total);
  return total;
}

size_t gemm_split3_workspace_size(int64_t m, int64_t n, int64_t k) {
  if (m < 0 || n < 0 || k < 0) return 0;
  int64_t kp, ldp;
  size_t off[6], total;
  split_layout(3, m, n, k, kp, ldp, off, total);
  return total;
}

static int split_convert(int np, int64_t rows, int64_t cols, const float *X, int64_t ldx,
                         int transpose, uint16_t *const *planes, int64_t ldo, void *stream) {
  clear_error();
  if (rows < 0 || cols < 0) return set_error(GEMM_EINVAL, "negative size");
  if (transpose != 0 && transpose != 1) return set_error(GEMM_EINVAL, "transpose must be 0 or 1");
  int rc;
  if ((rc = check_mat("X", X, rows, cols, ldx))) return rc;
  if (rows > 0 && cols > 0)
    for (int p = 0; p < np; ++p)
      if (planes[p] == nullptr) return set_error(GEMM_ENULL, "output plane is NULL");
  const int64_t out_cols = transpose ? rows : cols;
  if (ldo < out_cols) return set_error(GEMM_ELD, "ldo smaller than the plane row length");
  if (rows == 0 || cols == 0) return GEMM_OK;
  if ((rc = check_ld_range("X", ldx, 4))) return rc;
  hipError_t e = launch_split(np, rows, cols, X, ldx, transpose != 0, planes, ldo,
                              transpose ? rows : cols, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "split launch");
  return GEMM_OK;
}

int gemm_split_convert(int64_t rows, int64_t cols, const float *X, int64_t ldx, int transpose,
                       uint16_t *hi, uint16_t *lo, int64_t ldo, void *stream) {
  uint16_t *planes[2] = {hi, lo};
  return split_convert(2, rows, cols, X, ldx, transpose, planes, ldo, stream);
}

int gemm_split3_convert(int64_t rows, int64_t cols, const float *X, int64_t ldx, int transpose,
                        uint16_t *hi, uint16_t *mid, uint16_t *lo, int64_t ldo, void *stream) {
  uint16_t *planes[3] = {hi, mid, lo};
  return split_convert(3, rows, cols, X, ldx, transpose, planes, ldo, stream);
}

// The split product with np planes per operand: one split launch for both
// operands into the caller's workspace, then the product of the planes.
// The one-launch form of the split products (each fragment split in
// registers between the LDS read and the MFMAs) repeats the conversion in
// every wave that reads a fragment: it wins while the separate split step's
// launch and pass over A and B cost more than that, i.e. for products that
// leave most CUs idle and have a short K loop (N <= 1000: 1.2-1.6x faster;
// N = 1500: 7% slower, N = 2000: 18% slower, both precisions). It needs
// operands fit for 16-byte direct-to-LDS transfers.
//
// The loader form (one launch as well): loader waves split binary32 tiles
// once per workgroup into the LDS planes the compute waves read, so neither
// the planes' pass through device memory nor the per-wave repetition remain.
// It runs on the 128 x 128 loader-wave tile, one workgroup per CU. Measured
// (us, two-step against loader form): three-way split N = 1500 77.8 / 62.5,
// 2000 112.1 / 97.4, 2048 119.8 / 99.2, 2500 253.7 / 210.1, 3000 425.1 /
// 376.6, 4096 671.6 / 726.3; two-way split N = 1200 31.0 / 39.2, 2000 67.0 /
// 70.8, 2500 145.6 / 157.0, 4096 455.8 / 448.3 (the loaders' register loads
// of binary32 tiles keep pace with six products per tile, not with three).
// So the three-way split takes it from half a tile per CU to three tiles
// per CU, the two-way split keeps the two steps. With the plane products on
// the loader tile (choose_rule) a second sweep gave, nominal TFLOP/s: the
// two-way split in registers on the loader tile N = 1500 163 against 150
// (two steps), 1800 220 against 215, 2600 260 against 273; the three-way
// loader form N = 5000 176 against 161 (two steps, 128 x 256), 6144 197
// against 182, 8192 201 against 194, but N = 4096 193 against 207: the
// three-way split keeps the two steps from three to five tiles per CU.
// Up to one round of the loader tile the two-way split runs in registers:
// with operands read from HBM (each call after a 512 MiB fill, no sync) it
// took, us, N = 1800 61.4 against 61.9 for the two steps, 2000 66.7 against
// 71.3, 2048 66.5 against 73.9 (the product's own operand reads overlap its
// MFMAs, where the split step's pass over A and B does not); with operands
// that stay in the Infinity Cache from call to call (the same A and B back
// to back) the two steps are ahead at N = 2000 (61.9 against 65.9 us). From
// the second round on the forms are level (N = 2200 119.8 against 119.5,
// 2600 145.1 against 144.9) and the two steps stay.

static int split_form(int np, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                      const void *B, int64_t ldb) {
  const bool vec = vec_ok(A, lda, 4, k) && vec_ok(B, ldb, 4, n);
  const int lprec = np == 2 ? PREC_LSPLIT : PREC_LSPLIT3;
  const bool loaders = vec && plain_offered(lprec, LAYOUT_NN, CFG_128x128_K2_LD, 16);
  const int f = t_force_form;
  if (f == FORM_TWO_STEP) return FORM_TWO_STEP;
  if (f == FORM_REGISTERS) return vec ? FORM_REGISTERS : FORM_TWO_STEP;
  if (f == FORM_LOADERS) return loaders ? FORM_LOADERS : FORM_TWO_STEP;
  const int64_t t128 = ((m + 127) / 128) * ((n + 127) / 128);
  const int64_t cus = device_cus();
  if (vec && k <= 1024 && 2 * t128 <= cus) return FORM_REGISTERS;
  if (np == 2 && vec && 2 * t128 >= cus && t128 <= cus) return FORM_REGISTERS;
  if (np == 3 && loaders && 2 * t128 >= cus && (t128 < 3 * cus || t128 >= 5 * cus))
    return FORM_LOADERS;
  return FORM_TWO_STEP;
}

static bool split_one_launch(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                             const void *B, int64_t ldb) {
  return split_form(2, m, n, k, A, lda, B, ldb) == FORM_REGISTERS;
}

static int split_product(int np, int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                         const float *B, int64_t ldb, float *C, int64_t ldc, void *workspace,
                         size_t workspace_bytes, void *stream) {
  clear_error();
  if (m < 0 || n < 0 || k < 0) return set_error(GEMM_EINVAL, "negative size");
  int rc;
  if ((rc = check_mat("A", A, m, k, lda)) || (rc = check_mat("B", B, k, n, ldb)) ||
      (rc = check_mat("C", C, m, n, ldc)))
    return rc;
  if (m == 0 || n == 0) return GEMM_OK;
  int64_t kp, ldp;
  size_t off[6], total;
  split_layout(np, m, n, k, kp, ldp, off, total);
  if ((uint64_t)ldp * 2 >= kMaxPitch)
    return set_error(GEMM_EINVAL, "k too large (plane row pitch must be below 8 MiB)");
  if (workspace == nullptr || workspace_bytes < total)
    return set_error(GEMM_EWORKSPACE, "need " + std::to_string(total) + " bytes, got " +
                                          std::to_string(workspace_bytes));
  if ((uintptr_t)workspace % 16 != 0)
    return set_error(GEMM_EWORKSPACE, "workspace must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  // Small products and, two-way, up to one tile per CU: one launch that
  // splits each fragment in registers; three-way from half a tile per CU:
  // one launch whose loader waves split the tiles (both the same result bit
  // for bit as the two steps, no planes in device memory).
  const int form = split_form(np, m, n, k, A, lda, B, ldb);
  if (form == FORM_REGISTERS) {
    GemmArgs a{m, n, k, A, lda, B, ldb, nullptr, nullptr, C, ldc};
    return run_product(np == 2 ? PREC_FSPLIT : PREC_FSPLIT3, LAYOUT_NN, a, 4, s);
  }
  if (form == FORM_LOADERS) {
    if ((rc = check_ld_range("A", lda, 4)) || (rc = check_ld_range("B", ldb, 4))) return rc;
    GemmArgs a{m, n, k, A, lda, B, ldb, nullptr, nullptr, C, ldc};
    hipError_t e = launch_plain(np == 2 ? PREC_LSPLIT : PREC_LSPLIT3, LAYOUT_NN,
                                CFG_128x128_K2_LD, 16, a, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return GEMM_OK;
  }
  char *ws = (char *)workspace;
  uint16_t *ap[3] = {nullptr, nullptr, nullptr}, *bp[3] = {nullptr, nullptr, nullptr};
  for (int p = 0; p < np; ++p) {
    ap[p] = (uint16_t *)(ws + off[p]);
    bp[p] = (uint16_t *)(ws + off[np + p]);
  }
  if (k > 0) {
    // planes carry zeros in the padding columns [k, kp), so the product may
    // run over kp (a whole number of 8-element vectors) unchanged
    if ((rc = check_ld_range("A", lda, 4)) || (rc = check_ld_range("B", ldb, 4))) return rc;
    hipError_t e = launch_split_pair(np, m, n, k, A, lda, B, ldb, ap, bp, kp, ldp, s);
    if (e != hipSuccess) return hip_fail(e, "split launch");
  }
  GemmArgs a{m, n, k > 0 ? kp : 0, ap[0], ldp, bp[0], ldp, ap[1], bp[1], C, ldc, ap[2], bp[2]};
  return run_product(np == 2 ? PREC_SPLIT : PREC_SPLIT3, LAYOUT_NT, a, 2, s);
}

int gemm_split_one_launch(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                          const float *B, int64_t ldb) {
  clear_error();
  if (m <= 0 || n <= 0 || k < 0 || A == nullptr || B == nullptr) return 0;
  return split_one_launch(m, n, k, A, lda, B, ldb) ? 1 : 0;
}

int gemm_split(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B,
               int64_t ldb, float *C, int64_t ldc, void *workspace, size_t workspace_bytes,
               void *stream) {
  return split_product(2, m, n, k, A, lda, B, ldb, C, ldc, workspace, workspace_bytes, stream);
}

int gemm_split3(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B,
                int64_t ldb, float *C, int64_t ldc, void *workspace, size_t workspace_bytes,
                void *stream) {
  return split_product(3, m, n, k, A, lda, B, ldb, C, ldc, workspace, workspace_bytes, stream);
}

int gemm_backward(int dtype, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                  const void *B, int64_t ldb, const void *dC, int64_t lddc, void *dA,
                  int64_t ldda, void *dB, int64_t lddb, void *stream) {
  clear_error();
  if (dtype != GEMM_F64 && dtype != GEMM_F32 && dtype != GEMM_BF16)
    return set_error(GEMM_EUNSUPPORTED, "dtype " + std::to_string(dtype));
  if (m < 0 || n < 0 || k < 0) return set_error(GEMM_EINVAL, "negative size");
  int rc;
  if ((rc = check_mat("dC", dC, m, n, lddc))) return rc;
  if (dA && ((rc = check_mat("B", B, k, n, ldb)) || (rc = check_mat("dA", dA, m, k, ldda))))
    return rc;
  if (dB && ((rc = check_mat("A", A, m, k, lda)) || (rc = check_mat("dB", dB, k, n, lddb))))
    return rc;
  const int prec = dtype == GEMM_F64 ? PREC_F64 : dtype == GEMM_F32 ? PREC_F32 : PREC_BF16;
  const size_t es = esize_of(dtype);
  hipStream_t s = (hipStream_t)stream;
  if (dA) {  // dA (m x k) = dC (m x n) * B^T, B stored k x n: K-contiguous op(B)
    GemmArgs a{m, k, n, dC, lddc, B, ldb, nullptr, nullptr, dA, ldda};
    if ((rc = run_product(prec, LAYOUT_NT, a, es, s))) return rc;
  }
  if (dB) {  // dB (k x n) = A^T (k x m) * dC (m x n), A stored m x k
    GemmArgs a{k, n, m, A, lda, dC, lddc, nullptr, nullptr, dB, lddb};
    if ((rc = run_product(prec, LAYOUT_TN, a, es, s))) return rc;
  }
  return GEMM_OK;
}

}  // extern "C"
