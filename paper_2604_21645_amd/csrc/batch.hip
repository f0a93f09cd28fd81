// Batched fit + encode of many independent PQ problems (paper Section 3: the
// rows are split into chunks that are quantised in parallel).
//
// All problems advance together: each phase is ONE launch over every
// problem -- the persistent matrix-core assignment walks a flat list of
// (problem, subspace group, 32-row tile) units, the accumulation and the
// finalisation cover every (problem, chunk, subspace) item and every
// (problem, subspace) pair.  A plan fixes the assignment grid (optionally by
// timing candidates on the problems themselves) and can record the launch
// sequence as three HIP graphs: set-up, one Lloyd round (replayed `iters`
// times; the round index lives in device memory) and encode + error.
#include <errno.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "mipq_internal.h"

struct mipq_plan {
  std::vector<mipq_problem> probs;
  int d = 0, m = 0, ks = 0, iters = 0, precision = 0, flags = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int grid = 0;        // blocks of the persistent assignment
  int variant = 0;     // its register/occupancy variant
  int resident = 0;    // resident blocks of that variant on this device
  bool cached = false; // the choice came from the tuning cache
  bool fused = false;  // rounds run as one fused launch (its chunk layout)
  std::vector<int64_t> tried;   // (grid, variant, nanoseconds) per timed candidate
  hipGraphExec_t g_setup = nullptr, g_round = nullptr, g_final = nullptr;
};

namespace mipq {

namespace {

__global__ void k_copy_i64(const int64_t* __restrict__ src, int64_t* __restrict__ dst) {
  if (threadIdx.x == 0) dst[0] = src[0];
}

struct BatchLayout {
  BatchProb* probs = nullptr;   // device problem table
  uint32_t* round = nullptr;    // [0] round counter, [1] bad-init flag
  int64_t* resc = nullptr;      // pairs re-decided by the final encode
  double* c64 = nullptr;
  uint4* aop = nullptr;
  size_t aop_stride = 0;        // operand slots per problem
  float* cmax = nullptr;
  float* mu = nullptr;
  double* part_s = nullptr;
  uint32_t* part_cnt = nullptr;
  double* part_j = nullptr;
  double* j_all = nullptr;
  double* dpart = nullptr;
  float* tmax = nullptr;        // per-tile norm bounds of the finalize
  int64_t units = 0, items = 0, dblocks = 0;
  size_t bytes = 0;
};

// Work-list offsets of every problem (table may be NULL) and the workspace
// carving; the same code sizes and fills.
BatchLayout carve_batch(void* ws, const int64_t* n, int nprob, int d, int m, int ks, int iters,
                        std::vector<BatchProb>* table, const mipq_problem* probs, bool fused) {
  BatchLayout L;
  const int ds = d / m;
  const int groups = ceil_div(m, 4);
  if (table) table->resize(nprob);
  for (int p = 0; p < nprob; ++p) {
    const int64_t np = n[p];
    const int nch = fused ? fused_chunks(np) : update_chunks(np, m);
    const int nblk = decode_blocks(np, m);
    if (table) {
      BatchProb& b = (*table)[p];
      b.x = probs[p].x;
      b.n = np;
      b.init_rows = probs[p].init_rows;
      b.c32 = probs[p].codebook;
      b.codes = probs[p].codes;
      b.sse_rmse = probs[p].sse_rmse;
      b.objective = probs[p].objective;
      b.unit0 = L.units;
      b.item0 = L.items;
      b.rpc = (np + nch - 1) / nch;
      b.dblk0 = L.dblocks;
      b.nch = nch;
      b.nblk = nblk;
    }
    L.units += (int64_t)groups * ((np + 31) / 32);
    L.items += (int64_t)nch * m;
    L.dblocks += nblk;
  }
  Carver c(ws);
  const size_t per = (size_t)ks * ds;
  L.probs = c.take<BatchProb>(nprob);
  L.round = c.take<uint32_t>(4);
  L.resc = c.take<int64_t>(1);
  L.c64 = c.take<double>((size_t)nprob * m * per);
  L.aop_stride = bf16_operand_count(m, ks, ds);
  L.aop = c.take<uint4>((size_t)nprob * L.aop_stride);
  L.cmax = c.take<float>((size_t)nprob * m);
  L.mu = c.take<float>((size_t)nprob * m * kMaxDsBf16);
  L.part_s = c.take<double>((size_t)L.items * per);
  L.part_cnt = c.take<uint32_t>((size_t)L.items * ks);
  L.part_j = c.take<double>((size_t)L.items);
  L.j_all = c.take<double>((size_t)(iters > 0 ? iters : 1) * nprob * m);
  L.dpart = c.take<double>((size_t)L.dblocks);
  L.tmax = c.take<float>((size_t)nprob * m * kMaxTiles);
  L.bytes = c.bytes();
  return L;
}

int check_batch_shape(int nprob, int d, int m, int ks, int iters, int precision) {
  if (nprob < 1) return fail(MIPQ_EINVAL, "nprob must be >= 1 (got %d)", nprob);
  if (d <= 0 || m <= 0 || d % m) return fail(MIPQ_EINVAL, "d=%d must be a positive multiple of m=%d", d, m);
  if (ks < 1 || ks > kMaxKs) return fail(MIPQ_EINVAL, "ks must be in [1, %d] (got %d)", kMaxKs, ks);
  if (iters < 0 || iters > (1 << 16)) return fail(MIPQ_EINVAL, "iters out of range (%d)", iters);
  if (precision != MIPQ_BF16)
    return fail(MIPQ_EUNSUPPORTED, "batched fit runs the MIPQ_BF16 path only (got precision %d)", precision);
  if (d / m > kMaxDsBf16) return fail(MIPQ_EUNSUPPORTED, "batched fit supports d/m <= %d (got %d)", kMaxDsBf16, d / m);
  return MIPQ_OK;
}

int check_problems(const mipq_problem* probs, int nprob, int m) {
  if (!probs) return fail(MIPQ_EINVAL, "problem table is NULL");
  int64_t units = 0, blocks = 0;
  for (int p = 0; p < nprob; ++p) {
    const mipq_problem& q = probs[p];
    if (q.n < 1) return fail(MIPQ_EINVAL, "problem %d: n must be >= 1 (got %lld)", p, (long long)q.n);
    if ((uint64_t)q.n * (uint64_t)m >= (1ull << 32)) return fail(MIPQ_EUNSUPPORTED, "problem %d: n*m >= 2^32", p);
    if (!q.x || !q.init_rows || !q.codebook || !q.codes)
      return fail(MIPQ_EINVAL, "problem %d: x, init_rows, codebook and codes are required", p);
    units += (q.n + 31) / 32;
    blocks += std::max(update_chunks(q.n, m), fused_chunks(q.n)) * (int64_t)m;
  }
  if (units * ceil_div(m, 4) >= (1ll << 40) || blocks >= (1ll << 31))
    return fail(MIPQ_EUNSUPPORTED, "batched work list too long");
  return MIPQ_OK;
}

std::vector<int64_t> sizes_of(const mipq_problem* probs, int nprob) {
  std::vector<int64_t> n(nprob);
  for (int p = 0; p < nprob; ++p) n[p] = probs[p].n;
  return n;
}

struct BatchRun {
  BatchLayout L;
  int nprob, d, m, ks, iters;
  bool full, vec;
  int grid;
  bool det = false;   // MIPQ_PLAN_DETERMINISTIC
  int variant = 0;    // register/occupancy variant of the assignment
  bool obj = false;   // some problem returns its objective
  int fused_rpw = 0;  // > 0: rounds fuse the accumulation into the assignment
};

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

BatchRun make_run(const BatchLayout& L, const mipq_problem* probs, int nprob, int d, int m, int ks, int iters,
                  int grid, bool fused) {
  BatchRun r{L, nprob, d, m, ks, iters, true, true, grid, false, 0, false, 0};
  const int ds = d / m;
  const int nb = (ds + 7) / 8;
  r.full = (ds == nb * 8) && (d % 4 == 0);
  r.vec = ds % 4 == 0;
  for (int p = 0; p < nprob; ++p) {
    r.full = r.full && aligned16(probs[p].x);
    r.vec = r.vec && aligned16(probs[p].x) && aligned16(probs[p].codebook);
    r.obj = r.obj || probs[p].objective != nullptr;
  }
  r.fused_rpw = fused ? fit_round_batched_rpw(ks, ds, kFusedChunkRows) : 0;
  return r;
}

// Rounds fuse the accumulation into the assignment (chunks of fused_chunks
// rows) when no problem returns its objective, the sums need not be
// deterministic and a chunk's pending list fits a block's LDS.
bool batch_fused(const mipq_problem* probs, int nprob, int d, int m, int ks, bool det) {
  if (det) return false;
  for (int p = 0; p < nprob; ++p)
    if (probs[p].objective) return false;
  return fit_round_batched_rpw(ks, d / m, kFusedChunkRows) > 0;
}

// starting codebooks, round counter, operands of round 0
int run_setup(const BatchRun& r, hipStream_t s) {
  int rc;
  const BatchLayout& L = r.L;
  if ((rc = launch_zero_u32(L.round, 4, s))) return rc;
  if ((rc = launch_init_batched(L.probs, r.nprob, r.d, r.m, r.ks, L.c64, L.round + 1, s))) return rc;
  return launch_pack_bf16_batched(L.probs, r.nprob, r.m, r.ks, r.d / r.m, L.aop, L.aop_stride, L.cmax, L.mu, s);
}

// one Lloyd round of every problem: assign, accumulate (one fused launch
// when the plan allows it), finalise (+ pack)
int run_round(const BatchRun& r, hipStream_t s) {
  int rc;
  const BatchLayout& L = r.L;
  const bool fused = r.fused_rpw > 0;
  if (fused)
    rc = launch_fit_round_bf16_batched(L.probs, r.nprob, L.items, r.d, r.m, r.ks, L.aop, L.aop_stride, L.cmax, L.mu,
                                       r.full && r.vec, r.fused_rpw, L.part_s, L.part_cnt, L.part_j, s);
  else
    rc = launch_assign_bf16_batched(L.probs, r.nprob, L.units, r.d, r.m, r.ks, L.aop, L.aop_stride, L.cmax, L.mu,
                                    r.full, r.variant, r.grid, nullptr, s);
  if (rc) return rc;
  return launch_update_batched(L.probs, r.nprob, L.items, r.d, r.m, r.ks, L.c64, L.part_s, L.part_cnt, L.part_j,
                               L.j_all, L.round, r.iters, L.aop, L.aop_stride, L.cmax, L.mu, r.det, !fused, L.tmax,
                               s);
}

// encode with the final codebooks, reconstruction errors, objectives
int run_final(const BatchRun& r, hipStream_t s) {
  int rc;
  const BatchLayout& L = r.L;
  if ((rc = launch_zero_u32(reinterpret_cast<uint32_t*>(L.resc), 2, s))) return rc;
  if ((rc = launch_assign_bf16_batched(L.probs, r.nprob, L.units, r.d, r.m, r.ks, L.aop, L.aop_stride, L.cmax, L.mu,
                                       r.full, r.variant, r.grid, L.resc, s)))
    return rc;
  if ((rc = launch_decode_sse_batched(L.probs, r.nprob, L.dblocks, r.d, r.m, r.ks, r.vec, L.dpart, s))) return rc;
  return launch_objective_batched(L.probs, r.nprob, r.iters, r.m, L.j_all, s);
}

int upload_table(const BatchLayout& L, const std::vector<BatchProb>& table, hipStream_t s) {
  MIPQ_HIP(hipMemcpyAsync(L.probs, table.data(), table.size() * sizeof(BatchProb), hipMemcpyHostToDevice, s));
  MIPQ_HIP(hipStreamSynchronize(s));   // the host table is a local
  return MIPQ_OK;
}

int capture(hipStream_t cs, hipGraphExec_t* out, int (*fn)(const BatchRun&, hipStream_t), const BatchRun& r) {
  MIPQ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  const int rc = fn(r, cs);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  const hipError_t ei = hipGraphInstantiateWithFlags(out, g, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiateWithFlags");
  return MIPQ_OK;
}

void destroy_graphs(mipq_plan* p) {
  for (hipGraphExec_t* g : {&p->g_setup, &p->g_round, &p->g_final})
    if (*g) {
      (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
}

// ---- tuning cache ------------------------------------------------------------
// The plan's choice (grid multiple of the resident blocks, variant) per
// (device architecture, subspace width, ks, m, size bucket), kept in a JSON
// object (written one entry per line; read in any layout):
//   "gfx950:sramecc+:xnack-|ds=8|ks=256|m=12|rows=2^23|probs=2^6": {"grid_mult": 8, "variant": 0, "ns": 2781430},
// at $MIPQ_TUNE_CACHE, else $HOME/.cache/mipq/autotune.json.  Reading or
// writing it never fails a call: an unreadable cache is an empty one.
struct TuneEntry {
  int grid_mult = 0, variant = 0;
  long long ns = 0;
};

std::string tune_cache_path() {
  const char* e = getenv("MIPQ_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = getenv("HOME");
  return std::string(h && *h ? h : ".") + "/.cache/mipq/autotune.json";
}

int log2_bucket(int64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

std::string tune_key(int ds, int ks, int m, int64_t rows, int nprob) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|ds=%d|ks=%d|m=%d|rows=2^%d|probs=2^%d", arch.c_str(), ds, ks, m, log2_bucket(rows),
           log2_bucket(nprob));
  return buf;
}

// the integer after "name": inside [b, e), or false
bool json_int(const char* b, const char* e, const char* name, long long* out) {
  const std::string pat = std::string("\"") + name + "\"";
  const std::string obj(b, e);
  const size_t at = obj.find(pat);
  if (at == std::string::npos) return false;
  const char* p = obj.c_str() + at + pat.size();
  while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') ++p;
  if (*p++ != ':') return false;
  char* end = nullptr;
  errno = 0;
  const long long v = strtoll(p, &end, 10);
  if (end == p || errno) return false;
  *out = v;
  return true;
}

// entries "key": {"grid_mult": g, "variant": v, "ns": t} in any layout;
// anything else (or a damaged entry) is skipped
std::map<std::string, TuneEntry> tune_cache_read(const std::string& path) {
  std::map<std::string, TuneEntry> out;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return out;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0 && text.size() < (1u << 24)) text.append(buf, got);
  fclose(f);
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t kend = text.find('"', pos + 1);
    if (kend == std::string::npos) break;
    const std::string key = text.substr(pos + 1, kend - pos - 1);
    size_t q = kend + 1;
    while (q < text.size() && (text[q] == ' ' || text[q] == '\t' || text[q] == '\n' || text[q] == '\r')) ++q;
    if (q >= text.size() || text[q] != ':') {
      pos = kend + 1;
      continue;
    }
    ++q;
    while (q < text.size() && (text[q] == ' ' || text[q] == '\t' || text[q] == '\n' || text[q] == '\r')) ++q;
    if (q >= text.size() || text[q] != '{') {   // a field of an entry, not a key
      pos = q;
      continue;
    }
    const size_t close = text.find('}', q);
    if (close == std::string::npos) break;
    long long g = 0, v = 0, t = 0;
    const char* b = text.c_str() + q;
    const char* e = text.c_str() + close;
    if (json_int(b, e, "grid_mult", &g) && json_int(b, e, "variant", &v) && json_int(b, e, "ns", &t) && g >= 1 &&
        g <= 64 && v >= 0 && v < kBatchedVariants && t >= 0) {
      TuneEntry te;
      te.grid_mult = (int)g;
      te.variant = (int)v;
      te.ns = t;
      out[key] = te;
    }
    pos = close + 1;
  }
  return out;
}

void make_dirs(const std::string& path) {   // parents of path
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') {
      const std::string dir = path.substr(0, i);
      if (mkdir(dir.c_str(), 0755) != 0 && errno != EEXIST) return;
    }
}

void tune_cache_store(const std::string& path, const std::string& key, const TuneEntry& t) {
  std::map<std::string, TuneEntry> all = tune_cache_read(path);
  all[key] = t;
  make_dirs(path);
  const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : all)
    fprintf(f, " \"%s\": {\"grid_mult\": %d, \"variant\": %d, \"ns\": %lld}%s\n", kv.first.c_str(),
            kv.second.grid_mult, kv.second.variant, kv.second.ns, ++i < all.size() ? "," : "");
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), path.c_str()) != 0) remove(tmp.c_str());
}

bool same_problems(const mipq_problem* a, const std::vector<mipq_problem>& b, int nprob) {
  if ((int)b.size() != nprob) return false;
  return memcmp(a, b.data(), sizeof(mipq_problem) * nprob) == 0;
}

}  // namespace
}  // namespace mipq

using namespace mipq;

extern "C" {

size_t mipq_pq_fit_batched_workspace_size(const int64_t* n, int nprob, int d, int m, int ks, int iters,
                                          int precision) {
  if (!n || check_batch_shape(nprob, d, m, ks, iters, precision) != MIPQ_OK) return 0;
  for (int p = 0; p < nprob; ++p)
    if (n[p] < 1) return 0;
  // either chunk layout (fused rounds or not), whichever the plan takes
  return std::max(carve_batch(nullptr, n, nprob, d, m, ks, iters, nullptr, nullptr, false).bytes,
                  carve_batch(nullptr, n, nprob, d, m, ks, iters, nullptr, nullptr, true).bytes);
}

int mipq_plan_create(mipq_plan** out, const mipq_problem* probs, int nprob, int d, int m, int ks, int iters,
                     int precision, int flags, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if (!out) return fail(MIPQ_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if ((rc = check_batch_shape(nprob, d, m, ks, iters, precision))) return rc;
  if ((rc = check_problems(probs, nprob, m))) return rc;
  if (flags & ~(MIPQ_PLAN_AUTOTUNE | MIPQ_PLAN_GRAPH | MIPQ_PLAN_DETERMINISTIC | MIPQ_PLAN_RETUNE))
    return fail(MIPQ_EINVAL, "unknown plan flags 0x%x", flags);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::vector<int64_t> n = sizes_of(probs, nprob);
  std::vector<BatchProb> table;
  const bool fused = batch_fused(probs, nprob, d, m, ks, (flags & MIPQ_PLAN_DETERMINISTIC) != 0);
  const BatchLayout L = carve_batch(ws, n.data(), nprob, d, m, ks, iters, &table, probs, fused);
  if (!ws) return fail(MIPQ_EINVAL, "workspace pointer is NULL (%zu bytes needed)", L.bytes);
  if (ws_bytes < L.bytes) return fail(MIPQ_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, L.bytes);
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(MIPQ_EINVAL, "workspace must be 256-byte aligned");

  mipq_plan* plan = new mipq_plan;
  plan->fused = fused;
  plan->probs.assign(probs, probs + nprob);
  plan->d = d;
  plan->m = m;
  plan->ks = ks;
  plan->iters = iters;
  plan->precision = precision;
  plan->flags = flags;
  plan->ws = ws;
  plan->ws_bytes = ws_bytes;
  BatchRun r = make_run(L, probs, nprob, d, m, ks, iters, 8, fused);
  r.det = (flags & MIPQ_PLAN_DETERMINISTIC) != 0;
  auto bail = [&](int code) {
    destroy_graphs(plan);
    delete plan;
    return code;
  };
  // resident blocks of each variant, rounded up to whole XCD rounds (8)
  int res8[kBatchedVariants];
  for (int v = 0; v < kBatchedVariants; ++v) {
    int res = 0;
    if ((rc = assign_bf16_batched_resident(d / m, ks, r.full, v, &res))) return bail(rc);
    res8[v] = ((res > 8 ? res : 8) + 7) / 8 * 8;
  }
  plan->variant = 0;
  plan->grid = 2 * res8[0];
  if ((rc = upload_table(L, table, s))) return bail(rc);

  if (flags & MIPQ_PLAN_AUTOTUNE) {
    int64_t rows = 0;
    for (int64_t v : n) rows += v;
    const std::string path = tune_cache_path();
    const std::string key = tune_key(d / m, ks, m, rows, nprob);
    const std::map<std::string, TuneEntry> cache = (flags & MIPQ_PLAN_RETUNE) ? std::map<std::string, TuneEntry>()
                                                                              : tune_cache_read(path);
    const auto hit = cache.find(key);
    if (hit != cache.end()) {
      plan->variant = hit->second.variant;
      plan->grid = res8[plan->variant] * hit->second.grid_mult;
      plan->cached = true;
    } else {
      // time the assignment of round 0 (initial codebooks) for every variant
      // at a few grid sizes; the codes it writes are overwritten by the fit
      if ((rc = run_setup(r, s))) return bail(rc);
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return bail(fail(MIPQ_EHIP, "hipEventCreate failed"));
      }
      float best = 0.0f;
      int best_mult = 2;
      for (int v = 0; v < kBatchedVariants; ++v)
        for (int mult : {1, 2, 4, 8, 16}) {
          const int grid = res8[v] * mult;
          float ms = 0.0f;
          hipError_t e = hipSuccess;
          rc = launch_assign_bf16_batched(L.probs, nprob, L.units, d, m, ks, L.aop, L.aop_stride, L.cmax, L.mu,
                                          r.full, v, grid, nullptr, s);   // warm-up
          if (!rc && (e = hipEventRecord(a, s)) == hipSuccess) {
            for (int rep = 0; rep < 2 && !rc; ++rep)
              rc = launch_assign_bf16_batched(L.probs, nprob, L.units, d, m, ks, L.aop, L.aop_stride, L.cmax,
                                              L.mu, r.full, v, grid, nullptr, s);
            if (!rc && (e = hipEventRecord(b, s)) == hipSuccess && (e = hipEventSynchronize(b)) == hipSuccess)
              e = hipEventElapsedTime(&ms, a, b);
          }
          if (rc || e != hipSuccess) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            return bail(rc ? rc : hip_fail(e, "autotune timing"));
          }
          plan->tried.push_back(grid);
          plan->tried.push_back(v);
          plan->tried.push_back((int64_t)(ms * 0.5e6));
          if (best == 0.0f || ms < best) {
            best = ms;
            plan->grid = grid;
            plan->variant = v;
            best_mult = mult;
          }
        }
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      TuneEntry t;
      t.grid_mult = best_mult;
      t.variant = plan->variant;
      t.ns = (long long)(best * 0.5e6);
      tune_cache_store(path, key, t);
    }
  }
  plan->resident = res8[plan->variant];
  r.grid = plan->grid;
  r.variant = plan->variant;

  if (flags & MIPQ_PLAN_GRAPH) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(MIPQ_EHIP, "hipStreamCreateWithFlags failed"));
    rc = capture(cs, &plan->g_setup, run_setup, r);
    if (!rc) rc = capture(cs, &plan->g_round, run_round, r);
    if (!rc) rc = capture(cs, &plan->g_final, run_final, r);
    (void)hipStreamDestroy(cs);
    if (rc) return bail(rc);
  }
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
  *out = plan;
  return MIPQ_OK;
}

int mipq_plan_info(const mipq_plan* plan, int64_t* info, int count) {
  if (!plan || !info || count < 6) return fail(MIPQ_EINVAL, "plan and info[>= 6] are required");
  info[0] = plan->grid;
  info[1] = plan->resident;
  info[2] = plan->g_round != nullptr;
  info[3] = plan->variant;
  info[4] = plan->cached;
  info[5] = (int64_t)plan->tried.size() / 3;
  for (int i = 6; i < count; ++i) info[i] = (size_t)(i - 6) < plan->tried.size() ? plan->tried[i - 6] : 0;
  return MIPQ_OK;
}

int mipq_plan_destroy(mipq_plan* plan) {
  if (!plan) return MIPQ_OK;
  destroy_graphs(plan);
  delete plan;
  return MIPQ_OK;
}

int mipq_pq_fit_batched(const mipq_problem* probs, int nprob, int d, int m, int ks, int iters, int precision,
                        const mipq_plan* plan, int64_t* rescored, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_batch_shape(nprob, d, m, ks, iters, precision))) return rc;
  if ((rc = check_problems(probs, nprob, m))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::vector<int64_t> n = sizes_of(probs, nprob);
  if (plan) {
    if (plan->d != d || plan->m != m || plan->ks != ks || plan->iters != iters || plan->precision != precision ||
        !same_problems(probs, plan->probs, nprob))
      return fail(MIPQ_EINVAL, "the plan was made for other problems or shapes");
    if (plan->ws != ws || plan->ws_bytes > ws_bytes) return fail(MIPQ_EINVAL, "the plan was made for another workspace");
  }
  std::vector<BatchProb> table;
  const bool fused = plan ? plan->fused : batch_fused(probs, nprob, d, m, ks, false);
  const BatchLayout L = carve_batch(ws, n.data(), nprob, d, m, ks, iters, plan ? nullptr : &table, probs, fused);
  if (!ws) return fail(MIPQ_EINVAL, "workspace pointer is NULL (%zu bytes needed)", L.bytes);
  if (ws_bytes < L.bytes) return fail(MIPQ_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, L.bytes);
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(MIPQ_EINVAL, "workspace must be 256-byte aligned");
  if (plan && plan->g_round) {
    MIPQ_HIP(hipGraphLaunch(plan->g_setup, s));
    for (int it = 0; it < iters; ++it) MIPQ_HIP(hipGraphLaunch(plan->g_round, s));
    MIPQ_HIP(hipGraphLaunch(plan->g_final, s));
  } else {
    int grid = 0, variant = 0;
    if (plan) {
      grid = plan->grid;
      variant = plan->variant;
    } else {
      if ((rc = upload_table(L, table, s))) return rc;
      const int ds = d / m;
      int resident = 0;
      if ((rc = assign_bf16_batched_resident(ds, ks, make_run(L, probs, nprob, d, m, ks, iters, 8, fused).full, 0,
                                             &resident)))
        return rc;
      grid = 2 * (((resident > 8 ? resident : 8) + 7) / 8 * 8);
    }
    BatchRun r = make_run(L, probs, nprob, d, m, ks, iters, grid, fused);
    r.det = plan && (plan->flags & MIPQ_PLAN_DETERMINISTIC);
    r.variant = variant;
    if ((rc = run_setup(r, s))) return rc;
    for (int it = 0; it < iters; ++it)
      if ((rc = run_round(r, s))) return rc;
    if ((rc = run_final(r, s))) return rc;
  }
  if (rescored) {
    k_copy_i64<<<1, 64, 0, s>>>(L.resc, rescored);
    MIPQ_LAUNCHED("k_copy_i64");
  }
  return MIPQ_OK;
}

}  // extern "C"
