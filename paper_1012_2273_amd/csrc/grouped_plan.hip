// grouped_plan.hip -- host side of the grouped product: planner, tile-policy
// autotuner with a JSON cache, and hipGraph capture of the persistent launch.
//
// A policy assigns one tile configuration to each size class of problems
// (classes by max(m, n): <48, <96, <192, <384, <768, <1536, >=1536). The
// planner turns a policy into the device work list: every tile of every
// problem, in three queues (internal.h), each sorted by decreasing work (tile
// area x k), so that the persistent workgroups take the long tiles first and
// the short ones fill the tail.
// The tuner runs the persistent kernel on the caller's data for candidate
// policies (one class at a time, largest class first, every tile config)
// and keeps the fastest measured policy.
//
// Problems whose operands do not allow 16-byte transfers (binary64 rows of
// odd length, binary32 rows not a multiple of 4, unaligned bases) are packed
// unless the caller opts out: each run copies their A and B into plan-owned
// buffers with zero-padded, 16-byte rows (one launch for all of them, on a
// side stream beside the first queue's kernel, sized to finish under it),
// and the second queue's kernel reads those copies on the direct-to-LDS
// path instead of the register path's element loads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cctype>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "gemm_mi355x.h"
#include "gemm_tile.hpp"
#include "internal.h"

namespace g355 {

static constexpr int NCLASS = 7;
static const int64_t kClassEdge[NCLASS - 1] = {48, 96, 192, 384, 768, 1536};

static int size_class(int64_t m, int64_t n) {
  const int64_t s = std::max(m, n);
  int c = 0;
  while (c < NCLASS - 1 && s >= kClassEdge[c]) ++c;
  return c;
}

static const int kDefaultPolicy[NCLASS] = {CFG_32x32_K2, CFG_32x32_K2, CFG_64x64_K2,
                                           CFG_64x64_K2, CFG_64x64_K2, CFG_128x128_K2,
                                           CFG_128x128_K2};

// Last tuned policy per dtype in this process (used by gemm_grouped).
static std::mutex g_pol_mu;
static std::map<int, std::vector<int>> g_last_policy;

}  // namespace g355

struct gemm_plan {
  int dtype = 0;
  int prec = 0;
  int device = 0;
  std::vector<gemm_problem> probs;
  std::vector<g355::GroupedProblem> dprob_host;
  g355::GroupedProblem *d_probs = nullptr;
  g355::WorkItem *d_items = nullptr;
  uint32_t *d_counter = nullptr;
  int64_t items_cap = 0;
  int32_t n_items = 0;
  int32_t n_group[g355::kQueues] = {0, 0, 0};   // items per queue (see internal.h), in that order
  // packing: per problem the index of its A copy job (its B job follows), or -1
  std::vector<int32_t> pack_job;
  std::vector<g355::PackJob> jobs;
  g355::PackJob *d_jobs = nullptr;
  void *d_pack = nullptr;
  int64_t pack_blocks = 0;
  int pack_grid = 0;          // workgroups of the copy launch (see pack_grid_for)
  // the copies run on a side stream beside the first queue's kernel
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int grid = 0;
  int policy[g355::NCLASS];
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = false;
};

namespace g355 {

static int hip_fail(hipError_t e, const char *what) {
  return set_error(GEMM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Queue of a problem: 0 own operands with 16-byte rows, 1 packed, 2 register path.
static int queue_of(const gemm_plan &p, size_t i) {
  if (!p.pack_job.empty() && p.pack_job[i] >= 0) return 1;
  return p.dprob_host[i].vec ? 0 : 2;
}

static std::vector<WorkItem> plan_items(const gemm_plan &p, const int *policy,
                                        int32_t (&n_group)[kQueues]) {
  struct Keyed { int queue; int64_t cost; int64_t order; WorkItem w; };
  std::vector<Keyed> v;
  int64_t order = 0;
  for (size_t i = 0; i < p.probs.size(); ++i) {
    const gemm_problem &q = p.probs[i];
    if (q.m == 0 || q.n == 0) continue;
    const int cfg = policy[size_class(q.m, q.n)];
    const CfgInfo &ci = cfg_info(cfg);
    const int64_t tm = (q.m + ci.bm - 1) / ci.bm, tn = (q.n + ci.bn - 1) / ci.bn;
    const int64_t cost = (int64_t)ci.bm * ci.bn * std::max<int64_t>(q.k, 1);
    const int queue = queue_of(p, i);
    for (int64_t a = 0; a < tm; ++a)
      for (int64_t b = 0; b < tn; ++b)
        v.push_back({queue, cost, order++, WorkItem{(int32_t)i, cfg, (int32_t)a, (int32_t)b}});
  }
  // queue by queue, each largest work first
  std::stable_sort(v.begin(), v.end(), [](const Keyed &x, const Keyed &y) {
    if (x.queue != y.queue) return x.queue < y.queue;
    return x.cost > y.cost;
  });
  std::vector<WorkItem> out(v.size());
  for (int g = 0; g < kQueues; ++g) n_group[g] = 0;
  for (size_t i = 0; i < v.size(); ++i) {
    out[i] = v[i].w;
    n_group[v[i].queue]++;
  }
  return out;
}

static int upload_items(gemm_plan &p, const int *policy) {
  int32_t n_group[kQueues];
  std::vector<WorkItem> items = plan_items(p, policy, n_group);
  if ((int64_t)items.size() > 0x7fffffff) return set_error(GEMM_EINVAL, "too many tiles");
  if ((int64_t)items.size() > p.items_cap) return set_error(GEMM_ESTATE, "item capacity exceeded");
  if (!items.empty()) {
    hipError_t e = hipMemcpy(p.d_items, items.data(), items.size() * sizeof(WorkItem),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload work items");
  }
  p.n_items = (int32_t)items.size();
  std::memcpy(p.n_group, n_group, sizeof(n_group));
  std::memcpy(p.policy, policy, sizeof(p.policy));
  return GEMM_OK;
}

// Counter reset, then the three queues' kernels in order on `s`; the
// operand copies run on the side stream beside queue 0 and join `s` before
// queue 1 reads them. Captured as is, the fork and join become graph edges.
static int launch_direct(gemm_plan &p, hipStream_t s) {
  hipError_t e = launch_counter_reset(p.d_counter, s);
  const bool pack = !p.jobs.empty() && p.n_group[1] > 0;
  if (e == hipSuccess && pack) {
    e = hipEventRecord(p.ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(p.side, p.ev_fork, 0);
    if (e == hipSuccess)
      e = launch_pack(p.prec, p.d_jobs, (int32_t)p.jobs.size(), p.pack_blocks, p.pack_grid, p.side);
    if (e == hipSuccess) e = hipEventRecord(p.ev_join, p.side);
  }
  const WorkItem *it = p.d_items;
  for (int q = 0; q < kQueues && e == hipSuccess; ++q) {
    if (q == 1 && pack) e = hipStreamWaitEvent(s, p.ev_join, 0);
    if (e == hipSuccess)
      e = launch_grouped(p.prec, q < 2, p.d_probs, it, p.n_group[q],
                         p.d_counter + q * kCounterStride, p.grid, s);
    it += p.n_group[q];
  }
  if (e != hipSuccess) return hip_fail(e, "grouped launch");
  return GEMM_OK;
}

// ---------------------------------------------------------------- cache
// Format: a flat JSON object {"<key>": [c0, c1, ..., c6], ...}.
static std::map<std::string, std::vector<int>> cache_read(const char *path) {
  std::map<std::string, std::vector<int>> out;
  if (!path) return out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    const size_t lb = s.find('[', j), rb = s.find(']', j);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
    std::vector<int> vals;
    std::string body = s.substr(lb + 1, rb - lb - 1);
    for (char &ch : body)
      if (ch == ',') ch = ' ';
    std::stringstream bs(body);
    int x;
    while (bs >> x) vals.push_back(x);
    out[key] = vals;
    i = rb + 1;
  }
  return out;
}

static void cache_write(const char *path, const std::map<std::string, std::vector<int>> &m) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t n = 0;
    for (const auto &kv : m) {
      f << "  \"" << kv.first << "\": [";
      for (size_t i = 0; i < kv.second.size(); ++i) f << (i ? ", " : "") << kv.second[i];
      f << "]" << (++n < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

static std::string cache_key(const gemm_plan &p) {
  int hist[NCLASS] = {0};
  for (const auto &q : p.probs)
    if (q.m > 0 && q.n > 0) hist[size_class(q.m, q.n)]++;
  std::string key = p.dtype == GEMM_F64 ? "f64" : "f32";
  int dev_cus = 0;
  hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, p.device);
  key += "|cus" + std::to_string(dev_cus) + "|";
  for (int c = 0; c < NCLASS; ++c) key += (c ? "," : "") + std::to_string(hist[c]);
  return key;
}

static bool policy_valid(const std::vector<int> &v) {
  if ((int)v.size() != NCLASS) return false;
  for (int x : v)
    if (!cfg_grouped(x)) return false;
  return true;
}

// Time one policy: 1 warm-up + 3 timed runs, minimum in milliseconds.
static int time_policy(gemm_plan &p, const int *policy, hipStream_t s, float &ms_out) {
  int rc = upload_items(p, policy);
  if (rc) return rc;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return set_error(GEMM_EHIP, "event create");
  if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return set_error(GEMM_EHIP, "event create"); }
  float best = 1e30f;
  for (int r = 0; r < 4 && !rc; ++r) {
    hipEventRecord(e0, s);
    rc = launch_direct(p, s);
    hipEventRecord(e1, s);
    if (!rc) {
      hipError_t e = hipEventSynchronize(e1);
      if (e != hipSuccess) rc = hip_fail(e, "tuning run");
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) best = std::min(best, ms);
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  ms_out = best;
  return rc;
}

static int autotune(gemm_plan &p, hipStream_t s, int *policy) {
  bool present[NCLASS] = {false};
  for (const auto &q : p.probs)
    if (q.m > 0 && q.n > 0) present[size_class(q.m, q.n)] = true;
  float best_ms;
  int rc = time_policy(p, policy, s, best_ms);
  if (rc) return rc;
  for (int c = NCLASS - 1; c >= 0; --c) {
    if (!present[c]) continue;
    for (int cfg : kGroupedCfgs) {
      if (cfg == policy[c]) continue;
      int trial[NCLASS];
      std::memcpy(trial, policy, sizeof(trial));
      trial[c] = cfg;
      float ms;
      if ((rc = time_policy(p, trial, s, ms))) return rc;
      if (ms < best_ms * 0.99f) { best_ms = ms; policy[c] = cfg; }
    }
  }
  return GEMM_OK;
}

static int capture(gemm_plan &p) {
  hipStream_t cs;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "capture stream");
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) { hipStreamDestroy(cs); return hip_fail(e, "begin capture"); }
  int rc = launch_direct(p, cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  hipStreamDestroy(cs);
  if (rc) { if (g) hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) { hipGraphDestroy(g); return hip_fail(e, "graph instantiate"); }
  p.graph = g;
  p.exec = ex;
  return GEMM_OK;
}

static void plan_free(gemm_plan *p) {
  if (!p) return;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->d_probs) hipFree(p->d_probs);
  if (p->d_items) hipFree(p->d_items);
  if (p->d_counter) hipFree(p->d_counter);
  if (p->d_jobs) hipFree(p->d_jobs);
  if (p->d_pack) hipFree(p->d_pack);
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  if (p->ev_join) hipEventDestroy(p->ev_join);
  if (p->side) hipStreamDestroy(p->side);
  delete p;
}

static int validate_problems(int dtype, const gemm_problem *probs, int32_t count) {
  if (dtype != GEMM_F64 && dtype != GEMM_F32)
    return set_error(GEMM_EUNSUPPORTED, "grouped products take GEMM_F64 or GEMM_F32");
  if (count < 0) return set_error(GEMM_EINVAL, "negative count");
  if (count > 0 && probs == nullptr) return set_error(GEMM_ENULL, "problem array is NULL");
  for (int32_t i = 0; i < count; ++i) {
    const gemm_problem &q = probs[i];
    const std::string at = " (problem " + std::to_string(i) + ")";
    if (q.m < 0 || q.n < 0 || q.k < 0) return set_error(GEMM_EINVAL, "negative size" + at);
    if (q.m > 0x7fffffffLL * 32 || q.n > 0x7fffffffLL * 32)
      return set_error(GEMM_EINVAL, "size too large" + at);
    if (q.m > 0 && q.n > 0) {
      if (q.C == nullptr) return set_error(GEMM_ENULL, "C is NULL" + at);
      if (q.k > 0 && (q.A == nullptr || q.B == nullptr))
        return set_error(GEMM_ENULL, "A or B is NULL" + at);
    }
    if (q.lda < q.k || q.ldb < q.n || q.ldc < q.n)
      return set_error(GEMM_ELD, "leading dimension too small" + at);
    // the grouped shapes have at most 128 rows per operand tile: 32-bit tile
    // offsets stay below 2^31 for row pitches below 16 MiB
    const uint64_t es = dtype == GEMM_F64 ? 8 : 4;
    if ((uint64_t)q.lda * es >= (1ull << 24) || (uint64_t)q.ldb * es >= (1ull << 24))
      return set_error(GEMM_EINVAL, "leading dimension too large (row pitch must be below 16 MiB)" + at);
  }
  return GEMM_OK;
}

static GroupedProblem to_device(const gemm_problem &q, size_t es) {
  GroupedProblem d;
  d.M = q.m; d.N = q.n; d.K = q.k;
  d.A = q.A; d.B = q.B; d.C = q.C;
  d.lda = q.lda; d.ldb = q.ldb; d.ldc = q.ldc;
  // 16-byte loads: aligned bases and pitches, and K (A rows) and N (B rows)
  // whole numbers of vectors
  const int64_t v = 16 / (int64_t)es;
  d.vec = ((uintptr_t)q.A % 16 == 0) && ((uintptr_t)q.B % 16 == 0) &&
          ((uint64_t)q.lda * es % 16 == 0) && ((uint64_t)q.ldb * es % 16 == 0) &&
          (q.k % v == 0) && (q.n % v == 0);
  d.pad_ = 0;
  return d;
}

// Workgroups for the copies. They run beside the first queue's kernel (the
// problems with 16-byte rows of their own), which leaves room on every CU
// for a few copy workgroups; a full grid of them takes CU time and HBM from
// that kernel (binary64 512-problem batch: the first queue 4.38 ms alone,
// 5.02 beside 25398 copy workgroups). So the copies get just enough
// workgroups to finish within about three quarters of the first queue's
// estimated time: ~9 GB/s per copy workgroup beside the product (measured:
// 3.7 GB in 6.4 ms on 64), the first queue at 65 (binary64) / 120 (binary32)
// TFLOP/s. Measured replays (ms): binary64 10.77 with one workgroup per
// block, 10.17 with 128, 10.28 with 256, 12.17 with 64 (the copies then
// outlast the first queue); binary32 6.53 with one per block, 6.44 with
// 1024, 7.54 with 128.
static int pack_grid_for(const gemm_plan &p, size_t es) {
  double flops0 = 0.0, bytes = 0.0;
  for (size_t i = 0; i < p.probs.size(); ++i)
    if (p.pack_job[i] < 0 && p.dprob_host[i].vec)
      flops0 += 2.0 * (double)p.probs[i].m * (double)p.probs[i].n * (double)p.probs[i].k;
  for (const PackJob &j : p.jobs)
    bytes += (double)(j.rows * j.cols + j.drows * j.dcols) * (double)es;
  const double rate = p.prec == PREC_F64 ? 65e12 : 120e12;
  const double t0 = flops0 / rate;
  if (t0 <= 0.0) return 0;                     // nothing to hide under: one per block
  const double want = bytes / (0.75 * t0 * 9e9);
  const int64_t lo = std::min<int64_t>(64, p.pack_blocks);
  if (want >= (double)p.pack_blocks) return 0;
  return (int)std::max<int64_t>(lo, (int64_t)std::ceil(want));
}

// Lays out the packed copies of every problem whose operands do not allow
// 16-byte transfers (and whose product reads them: m, n, k > 0) in one
// device buffer and points those problems at them: A' = m x k' and B' =
// k' x n' with k', n' rounded up to whole vectors, zero padded, each copy
// 256-byte aligned. The problems then run with K = k' (the padding adds
// zero products) in the kernel of 16-byte transfers.
static int setup_packing(gemm_plan &p, size_t es) {
  const int64_t v = 16 / (int64_t)es;
  const size_t count = p.probs.size();
  p.pack_job.assign(count, -1);
  std::vector<std::pair<size_t, size_t>> off(count);
  size_t total = 0;
  auto take = [&](int64_t elems) {
    const size_t at = total;
    total += ((size_t)elems * es + 255) / 256 * 256;
    return at;
  };
  for (size_t i = 0; i < count; ++i) {
    const gemm_problem &q = p.probs[i];
    if (q.m == 0 || q.n == 0 || q.k == 0 || p.dprob_host[i].vec) continue;
    const int64_t kp = (q.k + v - 1) / v * v, np = (q.n + v - 1) / v * v;
    if ((uint64_t)kp * es >= (1ull << 24) || (uint64_t)np * es >= (1ull << 24))
      return set_error(GEMM_EINVAL, "packed row pitch too large (problem " + std::to_string(i) + ")");
    off[i].first = take(q.m * kp);
    off[i].second = take(kp * np);
    p.pack_job[i] = (int32_t)p.jobs.size();
    p.jobs.push_back(PackJob{q.A, nullptr, q.lda, kp, q.m, q.k, q.m, kp, 0});
    p.jobs.push_back(PackJob{q.B, nullptr, q.ldb, np, q.k, q.n, kp, np, 0});
  }
  if (p.jobs.empty()) return GEMM_OK;
  hipError_t e = hipMalloc(&p.d_pack, total);
  if (e == hipSuccess) e = hipMalloc(&p.d_jobs, sizeof(PackJob) * p.jobs.size());
  if (e != hipSuccess)
    return set_error(GEMM_ENOMEM, std::string("packed operand copies: ") + hipGetErrorString(e));
  e = hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p.ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p.ev_join, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "copy stream");
  char *base = static_cast<char *>(p.d_pack);
  int64_t blocks = 0;
  for (size_t i = 0; i < count; ++i) {
    if (p.pack_job[i] < 0) continue;
    PackJob &ja = p.jobs[p.pack_job[i]], &jb = p.jobs[p.pack_job[i] + 1];
    ja.dst = base + off[i].first;
    jb.dst = base + off[i].second;
    GroupedProblem &d = p.dprob_host[i];
    d.A = ja.dst; d.lda = ja.dld;
    d.B = jb.dst; d.ldb = jb.dld;
    d.K = ja.dcols;
    d.vec = 1;
  }
  for (PackJob &j : p.jobs) {
    j.first_block = blocks;
    blocks += (j.drows + kPackRows - 1) / kPackRows;
  }
  p.pack_blocks = blocks;
  p.pack_grid = pack_grid_for(p, es);
  e = hipMemcpy(p.d_jobs, p.jobs.data(), sizeof(PackJob) * p.jobs.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload copy jobs");
  return GEMM_OK;
}

}  // namespace g355

using namespace g355;

extern "C" {

int gemm_grouped_plan_create(gemm_plan **out, int dtype, const gemm_problem *probs,
                             int32_t count, const char *tune_cache, int flags, void *stream) {
  clear_error();
  if (!out) return set_error(GEMM_ENULL, "out is NULL");
  *out = nullptr;
  if (flags & ~(GEMM_PLAN_AUTOTUNE | GEMM_PLAN_NO_GRAPH | GEMM_PLAN_NO_PACK))
    return set_error(GEMM_EINVAL, "unknown plan flags");
  int rc = validate_problems(dtype, probs, count);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;

  gemm_plan *p = new (std::nothrow) gemm_plan();
  if (!p) return set_error(GEMM_ENOMEM, "plan");
  p->dtype = dtype;
  p->prec = dtype == GEMM_F64 ? PREC_F64 : PREC_F32;
  hipGetDevice(&p->device);
  p->probs.assign(probs, probs + count);
  const size_t es = dtype == GEMM_F64 ? 8 : 4;
  p->dprob_host.resize(count);
  p->pack_job.assign(count, -1);
  int64_t cap = 0;
  for (int32_t i = 0; i < count; ++i) {
    p->dprob_host[i] = to_device(probs[i], es);
    if (probs[i].m > 0 && probs[i].n > 0) {
      int64_t worst = 0;   // most tiles any configuration can produce
      for (int c : kGroupedCfgs) {
        const CfgInfo &ci = cfg_info(c);
        worst = std::max(worst, ((probs[i].m + ci.bm - 1) / ci.bm) * ((probs[i].n + ci.bn - 1) / ci.bn));
      }
      cap += worst;
    }
  }
  p->items_cap = cap;
  if (!(flags & GEMM_PLAN_NO_PACK) && (rc = setup_packing(*p, es))) { plan_free(p); return rc; }
  hipError_t e = hipSuccess;
  if (count > 0) e = hipMalloc(&p->d_probs, sizeof(GroupedProblem) * count);
  if (e == hipSuccess && cap > 0) e = hipMalloc(&p->d_items, sizeof(WorkItem) * cap);
  if (e == hipSuccess) e = hipMalloc(&p->d_counter, sizeof(uint32_t) * 64);
  if (e != hipSuccess) {
    plan_free(p);
    return set_error(GEMM_ENOMEM, std::string("plan device arrays: ") + hipGetErrorString(e));
  }
  if (count > 0)
    e = hipMemcpy(p->d_probs, p->dprob_host.data(), sizeof(GroupedProblem) * count,
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) { plan_free(p); return hip_fail(e, "upload problems"); }
  p->grid = grouped_max_grid(p->prec);
  if (p->grid <= 0) { plan_free(p); return set_error(GEMM_EHIP, "occupancy query failed"); }

  // policy: cache hit > tuning > last tuned in this process > default
  int policy[NCLASS];
  std::memcpy(policy, kDefaultPolicy, sizeof(policy));
  {
    std::lock_guard<std::mutex> lk(g_pol_mu);
    auto it = g_last_policy.find(dtype);
    if (it != g_last_policy.end()) std::copy(it->second.begin(), it->second.end(), policy);
  }
  const std::string key = cache_key(*p);
  auto cache = cache_read(tune_cache);
  bool have = false;
  auto hit = cache.find(key);
  if (hit != cache.end() && policy_valid(hit->second)) {
    std::copy(hit->second.begin(), hit->second.end(), policy);
    have = true;
  }
  if ((flags & GEMM_PLAN_AUTOTUNE) && !have) {
    if ((rc = autotune(*p, s, policy))) { plan_free(p); return rc; }
    cache[key] = std::vector<int>(policy, policy + NCLASS);
    cache_write(tune_cache, cache);
    std::lock_guard<std::mutex> lk(g_pol_mu);
    g_last_policy[dtype] = std::vector<int>(policy, policy + NCLASS);
  }
  if ((rc = upload_items(*p, policy))) { plan_free(p); return rc; }
  if (!(flags & GEMM_PLAN_NO_GRAPH)) {
    if ((rc = capture(*p))) { plan_free(p); return rc; }
    p->use_graph = true;
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) { plan_free(p); return hip_fail(e, "plan synchronise"); }
  *out = p;
  return GEMM_OK;
}

int gemm_grouped_run(gemm_plan *plan, void *stream) {
  clear_error();
  if (!plan) return set_error(GEMM_ENULL, "plan is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (plan->use_graph) {
    hipError_t e = hipGraphLaunch(plan->exec, s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return GEMM_OK;
  }
  return launch_direct(*plan, s);
}

int gemm_grouped_plan_update(gemm_plan *plan, const gemm_problem *probs, int32_t count) {
  clear_error();
  if (!plan || (!probs && count > 0)) return set_error(GEMM_ENULL, "plan or problems NULL");
  if (count != (int32_t)plan->probs.size()) return set_error(GEMM_EINVAL, "count differs");
  const size_t es = plan->dtype == GEMM_F64 ? 8 : 4;
  for (int32_t i = 0; i < count; ++i) {
    const gemm_problem &o = plan->probs[i], &q = probs[i];
    if (o.m != q.m || o.n != q.n || o.k != q.k || o.lda != q.lda || o.ldb != q.ldb ||
        o.ldc != q.ldc)
      return set_error(GEMM_EINVAL, "shape differs at problem " + std::to_string(i));
    if (q.m > 0 && q.n > 0 && (q.C == nullptr || (q.k > 0 && (!q.A || !q.B))))
      return set_error(GEMM_ENULL, "NULL matrix at problem " + std::to_string(i));
    // the captured work list runs each problem in the kernel its planned
    // operands allowed: a problem planned with 16-byte transfers of the
    // caller's operands keeps them, so its new A and B must allow them too
    // (a packed problem's copies take any alignment)
    if (plan->pack_job[i] < 0 && plan->dprob_host[i].vec && !to_device(q, es).vec)
      return set_error(GEMM_EINVAL, "problem " + std::to_string(i) +
                                        " was planned with 16-byte aligned operands; the new A or "
                                        "B is not 16-byte aligned");
  }
  // new device records first; the plan takes them once both uploads succeed
  std::vector<GroupedProblem> dprob = plan->dprob_host;
  std::vector<PackJob> jobs = plan->jobs;
  for (int32_t i = 0; i < count; ++i) {
    const int32_t pj = plan->pack_job[i];
    if (pj >= 0) {   // the copies stay; their sources and C move
      jobs[pj].src = probs[i].A;
      jobs[pj + 1].src = probs[i].B;
      dprob[i].C = probs[i].C;
    } else {
      const int32_t planned = dprob[i].vec;
      dprob[i] = to_device(probs[i], es);
      dprob[i].vec = planned;   // the work list's split stays as captured
    }
  }
  if (count > 0) {
    hipError_t e = hipMemcpy(plan->d_probs, dprob.data(), sizeof(GroupedProblem) * count,
                             hipMemcpyHostToDevice);
    if (e == hipSuccess && !jobs.empty())
      e = hipMemcpy(plan->d_jobs, jobs.data(), sizeof(PackJob) * jobs.size(),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      // put the device records back as they were, so that nothing changes
      hipMemcpy(plan->d_probs, plan->dprob_host.data(), sizeof(GroupedProblem) * count,
                hipMemcpyHostToDevice);
      if (!plan->jobs.empty())
        hipMemcpy(plan->d_jobs, plan->jobs.data(), sizeof(PackJob) * plan->jobs.size(),
                  hipMemcpyHostToDevice);
      return hip_fail(e, "upload problems");
    }
  }
  plan->probs.assign(probs, probs + count);
  plan->dprob_host.swap(dprob);
  plan->jobs.swap(jobs);
  return GEMM_OK;
}

int gemm_grouped_plan_destroy(gemm_plan *plan) {
  clear_error();
  plan_free(plan);
  return GEMM_OK;
}

int gemm_grouped_plan_info(const gemm_plan *plan, int64_t *tiles, int32_t *policy, int32_t cap) {
  clear_error();
  if (!plan) return set_error(GEMM_ENULL, "plan is NULL");
  if (tiles) *tiles = plan->n_items;
  if (policy)
    for (int32_t i = 0; i < cap && i < NCLASS; ++i) policy[i] = plan->policy[i];
  return GEMM_OK;
}

int gemm_grouped(int dtype, const gemm_problem *probs, int32_t count, void *stream) {
  gemm_plan *p = nullptr;
  int rc = gemm_grouped_plan_create(&p, dtype, probs, count, nullptr, GEMM_PLAN_NO_GRAPH, stream);
  if (rc) return rc;
  rc = gemm_grouped_run(p, stream);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  plan_free(p);
  if (!rc && e != hipSuccess) rc = hip_fail(e, "grouped synchronise");
  return rc;
}

}  // extern "C"
