// Host runtime: argument checks, workspace planning, launch sequence and the
// C-ABI entry points (see include/etest.h).
#include "runtime.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace et {

static thread_local std::string g_err;

etest_status set_error(etest_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_OK(call, what)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_error(ETEST_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_));     \
  } while (0)

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static int env_int(const char* name, int dflt, int lo, int hi) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  int x = atoi(v);
  return x < lo ? lo : (x > hi ? hi : x);
}

etest_status validate_request(const etest_request& r) {
  if (r.kind != ETEST_ED && r.kind != ETEST_MMD) return set_error(ETEST_EINVAL, "kind must be ED or MMD");
  if (r.prec != ETEST_PREC_F64 && r.prec != ETEST_PREC_F32 && r.prec != ETEST_PREC_BF16_REFINED)
    return set_error(ETEST_EINVAL, "unknown precision");
  if (r.nx < 1 || r.ny < 1) return set_error(ETEST_EINVAL, "nx and ny must be >= 1");
  if (r.p < 1) return set_error(ETEST_EINVAL, "p must be >= 1");
  if (r.B < 0) return set_error(ETEST_EINVAL, "B must be >= 0");
  if (r.nx + r.ny > 2147483647LL) return set_error(ETEST_EINVAL, "nx + ny must be < 2^31");
  // ny = 0 only for the one-sample plans of the HSIC test (never a two-sample request)
  const int64_t nt = (r.nx + TILE - 1) / TILE + (r.ny + TILE - 1) / TILE;
  if (nt > MAX_TILE_GRID)
    return set_error(ETEST_EINVAL, "nx + ny too large for one test: " + std::to_string(nt) +
                                       " pooled tiles of 128 rows, at most " +
                                       std::to_string(MAX_TILE_GRID));
  if (r.p > 2147483647LL / 2) return set_error(ETEST_EINVAL, "p too large");
  if (r.B > 2147483646LL) return set_error(ETEST_EINVAL, "B must be < 2^31 - 1");
  if (r.kind == ETEST_MMD && !(std::isfinite(r.gamma) && r.gamma > 0.0))
    return set_error(ETEST_EINVAL, "gamma must be finite and > 0");
  if (!r.X || !r.Y) return set_error(ETEST_EINVAL, "X and Y must not be NULL");
  return ETEST_OK;
}


// ------------------------------------------------------------------ tuning rules
struct TuneRule {
  int32_t prec;
  int64_t n_lo, n_hi;
  int32_t kc, cc;
};
struct GramRule {
  int32_t prec;
  int64_t n_lo, n_hi;
  int32_t shape;
};
static std::mutex g_tune_mu;
static std::vector<TuneRule> g_tune;
static std::vector<GramRule> g_tune_gram;
static uint64_t g_tune_gen = 0;  // bumped on every change (guarded by g_tune_mu)

static uint64_t tune_generation() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tune_gen;
}

// Resampling work shape for a test: (column tiles per workgroup, chunks per workgroup).
// Without a tuned rule: 16 column tiles per workgroup (each workgroup's start-up -- its
// first tile load and the fold at the end -- is paid once per unit), halved while the
// launch would have fewer than 512 workgroups (two per CU), so small tests still spread
// over the chip.
static void tuned_shape(const etest_request& r, int32_t* kc, int32_t* cc) {
  // the FP64 kernel stages its strip again for every chunk, so grouping chunks in one
  // workgroup only serialises them: one chunk per workgroup
  *cc = r.prec == ETEST_PREC_F64 ? 1 : 2;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int64_t n = r.nx + r.ny;
    for (const TuneRule& t : g_tune)
      if (t.prec == r.prec && n >= t.n_lo && n < t.n_hi) {
        *kc = t.kc;
        *cc = t.cc;
        return;
      }
  }
  const int64_t nt = (r.nx + TILE - 1) / TILE + (r.ny + TILE - 1) / TILE;
  const int64_t chunks = (r.B + 1 + NP - 1) / NP;
  const int64_t ncr = (chunks + *cc - 1) / *cc;
  // the FP64 kernel runs PC_STRIPS workgroups per row unit and may go down to one tile each
  const bool f64 = r.prec == ETEST_PREC_F64;
  const int64_t strips = f64 ? PC_STRIPS : 1;
  // MFMA forms on 64 tiles or more: longer row units (measured on 5000 + 4000 pooled rows:
  // 5% (BF16-refined) and 9% (FP32) less resampling time than 16 tiles per unit)
  *kc = (!f64 && nt >= 64) ? 64 : 16;
  while (*kc > (f64 ? 1 : 2)) {
    int64_t nrk = 0;
    for (int64_t i = 0; i < nt; ++i) nrk += (nt - i + *kc - 1) / *kc;
    if (nrk * strips * ncr >= 512) break;
    *kc /= 2;
  }
}

// Workgroups of the super-tile Gram: the upper triangle of the ceil(nt / 2) super grid.
static int64_t super_tiles(int64_t nt) {
  const int64_t st = (nt + 1) / 2;
  return st * (st + 1) / 2;
}

// Gram workgroup shape of a test: a tuned rule for its precision and pooled size, else
// super tiles (2 x 2 stored tiles per workgroup) once there are at least
// GRAM_SUPER_MIN_WG of them -- two rounds of the 256 CUs, as a super-tile workgroup holds
// a CU alone -- and 128-tile workgroups below.  FP64 blocks have one shape.
constexpr int64_t GRAM_SUPER_MIN_WG = 512;
static int gram_shape(const etest_request& r, int64_t nt) {
  if (r.prec == ETEST_PREC_F64) return GSHAPE_TILE;
  // the super-tile kernel forms its staged-row offsets within a tile in 32 bits
  if ((r.p + 64) * 4 * (int64_t)TILE >= (int64_t)1 << 31) return GSHAPE_TILE;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int64_t n = r.nx + r.ny;
    for (const GramRule& g : g_tune_gram)
      if (g.prec == r.prec && n >= g.n_lo && n < g.n_hi) return g.shape;
  }
  const int env = env_int("ETEST_GRAM_SHAPE", -1, -1, 1);
  if (env >= 0) return env;
  return super_tiles(nt) >= GRAM_SUPER_MIN_WG ? GSHAPE_SUPER : GSHAPE_TILE;
}

TestPlan make_plan(const etest_request& r, int64_t kc_override, int mode) {
  TestPlan P;
  TestDesc& d = P.d;
  d.kind = r.kind;
  d.prec = r.prec;
  d.nx = (int32_t)r.nx;
  d.ny = (int32_t)r.ny;
  d.p = (int32_t)r.p;
  d.gop = gram_operands(r.prec, r.p);
  const int kq = gram_k_slice(d.gop);
  d.p_pad = (int32_t)((r.p + kq - 1) / kq * kq);
  d.tx = (int32_t)((r.nx + TILE - 1) / TILE);
  d.ty = (int32_t)((r.ny + TILE - 1) / TILE);
  d.nt = d.tx + d.ty;
  // below 2^31 for every grid validate_request accepts (nt <= MAX_TILE_GRID), the dense
  // nt x nt grid included (46340^2 < 2^31)
  const bool precomp = mode == PLAN_PRECOMP || mode == PLAN_PRECOMP_DENSE;
  d.dense = mode == PLAN_PRECOMP_DENSE ? 1 : 0;
  d.ntiles = (int32_t)(d.dense ? (int64_t)d.nt * d.nt : (int64_t)d.nt * (d.nt + 1) / 2);
  // fp16 planes of the centred blocks: hi + lo 2^-11 keeps ~22 significant bits of each
  // centred entry.  One plane (11 bits) is not enough even for the BF16 form: a statistic
  // is a sum with heavy cancellation, and on small tests 11-bit entries move it by ~1e-3.
  d.pfmt = r.prec == ETEST_PREC_F64 ? 0
           : r.prec == ETEST_PREC_F32 ? PLANES_F16_F16 : PLANES_F16_E4M3;
  d.refine = r.prec == ETEST_PREC_F64 ? 0 : 1;
  int32_t kc_t, cc_t;
  tuned_shape(r, &kc_t, &cc_t);
  d.kc = (int32_t)(kc_override > 0 ? kc_override : kc_t);
  int64_t nrk = 0;
  for (int64_t i = 0; i < d.nt; ++i) nrk += (d.nt - i + d.kc - 1) / d.kc;
  if (r.prec == ETEST_PREC_F64) nrk *= PC_STRIPS;  // FP64: one unit per strip
  // a count past 2^31 - 1 (tiny row units on a huge grid) is saturated here and rejected by
  // check_launch_sizes
  d.n_rowk = (int32_t)std::min<int64_t>(nrk, 2147483647LL);
  const int64_t n = r.nx + r.ny;
  d.nrowchunks = (int32_t)((n + COLSUM_ROWS - 1) / COLSUM_ROWS);
  d.B = r.B;
  d.B_pad = (r.B + 1 + NP - 1) / NP * NP;
  // split chunks per resampling workgroup: the MFMA kernel holds two accumulator sets
  const int cc_max = r.prec == ETEST_PREC_F64 ? MAX_CC : 2;
  d.cc = (int32_t)std::min<int64_t>(std::min(env_int("ETEST_CC", cc_t, 1, MAX_CC), cc_max),
                                    d.B_pad / NP);
  d.seed = r.seed;
  d.gamma = r.kind == ETEST_MMD ? r.gamma : 0.0;
  d.X = r.X;
  d.Y = r.Y;
  d.perm_out = r.perm_stats;

  const bool f64 = r.prec == ETEST_PREC_F64;
  const int64_t npad = (int64_t)d.nt * TILE;
  const size_t el_w = (size_t)gram_operand_bytes(d.gop);
  const size_t el_d = f64 ? 8 : 4;
  size_t sz[B_NBUF] = {};
  sz[B_COLPART] = f64 ? 0 : (size_t)d.nrowchunks * r.p * 8;
  sz[B_COLMEAN] = f64 ? 0 : (size_t)r.p * 8;
  sz[B_W] = (size_t)npad * d.p_pad * el_w;
  sz[B_NRM] = (size_t)npad * (f64 ? 8 : 4);
  sz[B_D] = (size_t)d.ntiles * TILE * TILE * el_d;
  sz[B_TSUM] = (size_t)d.ntiles * TSUM_STRIDE * 8;
  sz[B_TMAX] = (size_t)d.ntiles * TMAX_PER_TILE * 4;
  sz[B_RSUM] = (size_t)npad * 2 * 8;
  sz[B_OBS] = 8 * 8;
  sz[B_PLANES] = f64 ? (size_t)d.ntiles * TILE * TILE * 8
                     : (size_t)d.ntiles * TILE * TILE * plane_bytes_per_entry(d.pfmt);
  sz[B_Z] = (size_t)(npad / 32) * d.B_pad * 4;
  sz[B_PART] = (size_t)d.n_rowk * d.B_pad * 8;
  sz[B_PSTAT] = (size_t)d.B_pad * 8;
  sz[B_FLAGS] = FLAG_WORDS * 4;
  sz[B_RESULT] = sizeof(DevResult);
  sz[B_PERMOUT] = 0;  // set by build_batch when an internal output is needed
  if (mode != PLAN_EFFICIENT) {  // no centred planes or resampling buffers
    sz[B_PLANES] = 0;
    sz[B_PART] = 0;
    sz[B_PSTAT] = 0;
    if (mode == PLAN_BLOCKS) sz[B_Z] = 0;
    if (precomp) {
      sz[B_PART] = (size_t)d.ntiles * PC_STRIPS * 3 * d.B_pad * 8;
      sz[B_PSTAT] = (size_t)d.B_pad * 8;
    }
  }
  size_t o = 0;
  for (int k = 0; k < B_PERMOUT; ++k) {
    P.off[k] = o;
    P.size[k] = sz[k];
    o += align256(sz[k]);
  }
  P.bytes = o;
  P.internal_perm = false;  // build_batch appends an internal output buffer when asked

  const bool f32like = !f64;
  P.wg[S_COLPART] = f32like ? colpart_wgs(d.nrowchunks, r.p) : 0;
  P.wg[S_COLMEAN] = f32like ? (r.p + 63) / 64 : 0;
  P.wg[S_STAGE] = stage_wgs(npad, d.p_pad);
  // the dense grid keeps one 128-tile workgroup per tile
  d.gshape = d.dense ? GSHAPE_TILE : gram_shape(r, d.nt);
  const bool sup = d.gshape == GSHAPE_SUPER;
  P.wg[S_GRAM_F64] = f64 ? d.ntiles : 0;
  P.wg[S_GRAM_F32] = d.gop == GOP_F16PAIR && !sup ? d.ntiles : 0;
  P.wg[S_GRAM_BF16] = d.gop == GOP_BF16 && !sup ? d.ntiles : 0;
  P.wg[S_GRAM_F32S] = d.gop == GOP_F16PAIR && sup ? super_tiles(d.nt) : 0;
  P.wg[S_GRAM_BF16S] = d.gop == GOP_BF16 && sup ? super_tiles(d.nt) : 0;
  P.wg[S_GRAM_FIN] = sup ? d.ntiles : 0;
  P.wg[S_MEMBER] = d.B_pad / MEMBER_SPLITS;
  P.wg[S_ROWSUM] = (2 * npad + 63) / 64;  // two threads per pooled position
  P.wg[S_CENTER_F64] = f64 ? d.ntiles : 0;
  // one workgroup per half tile, or per tile on grids past 2^22 tiles (one dispatch holds
  // fewer than 2^32 work-items)
  P.wg[S_CENTER_SPLIT] = f64 ? 0 : (int64_t)d.ntiles * (d.ntiles <= (1 << 22) ? 2 : 1);
  const int64_t perm_wg = perm_units(d, (int)(d.B_pad / NP));
  P.wg[S_PERM_F64] = f64 ? perm_wg : 0;
  P.wg[S_PERM_S2] = d.pfmt == PLANES_F16_F16 ? perm_wg : 0;
  P.wg[S_PERM_S3] = d.pfmt == PLANES_F16_E4M3 ? perm_wg : 0;
  P.wg[S_PSTAT] = d.B_pad / 64;
  if (mode != PLAN_EFFICIENT)
    for (int k : {S_CENTER_F64, S_CENTER_SPLIT, S_PERM_F64, S_PERM_S2, S_PERM_S3, S_PSTAT})
      P.wg[k] = 0;
  if (mode == PLAN_BLOCKS) P.wg[S_MEMBER] = 0;
  if (precomp) P.wg[S_ROWSUM] = 0;
  return P;
}

Pairing pair_tests(const etest_request* reqs, int64_t n) {
  Pairing P;
  P.partner.assign((size_t)n, -1);
  P.share_z.assign((size_t)n, 0);
  std::vector<char> fed((size_t)n, 0);
  for (int64_t s = 0; s < n; ++s) {
    const etest_request& a = reqs[s];
    if (a.kind != ETEST_ED || a.prec == ETEST_PREC_F64) continue;
    for (int64_t u = 0; u < n; ++u) {
      const etest_request& m = reqs[u];
      if (fed[(size_t)u] || m.kind != ETEST_MMD || m.prec != a.prec || m.X != a.X ||
          m.Y != a.Y || m.nx != a.nx || m.ny != a.ny || m.p != a.p)
        continue;
      P.partner[(size_t)s] = (int)u;
      P.share_z[(size_t)s] = (char)(m.seed == a.seed && m.B == a.B);
      fed[(size_t)u] = 1;
      break;
    }
  }
  return P;
}

void link_partners(TestDesc* descs, const Pairing& pairing) {
  for (size_t s = 0; s < pairing.partner.size(); ++s) {
    TestDesc& a = descs[s];
    a.pD = nullptr;
    a.ptsum = nullptr;
    a.ptmax = nullptr;
    a.pflags = nullptr;
    a.pgamma = 0.0;
    const int u = pairing.partner[s];
    if (u < 0) continue;
    TestDesc& m = descs[u];
    a.pD = m.D;
    a.ptsum = m.tsum;
    a.ptmax = m.tmax;
    a.pflags = m.flags;
    a.pgamma = m.gamma;
    if (pairing.share_z[s]) m.Z = a.Z;  // identical split streams: one copy
  }
}

// Threads per workgroup of each launch slot.
static int slot_threads(int s) {
  switch (s) {
    case S_COLMEAN: return 64 * CM_GROUPS;
    case S_MEMBER: return MTHREADS;
    case S_ROWSUM: return 64;
    case S_PERM_S2:
    case S_PERM_S3: return PERM_THREADS;
    case S_PSTAT: return 64 * PS_GROUPS;
    default: return 256;
  }
}

// Every launch of a batch is one flattened grid per slot: its workgroup count must stay
// below 2^31 (workgroup indices are formed in 32 bits) and its work-item count below 2^32
// (the dispatch's grid size); a test's row units must stay below 2^31 as well.
etest_status check_launch_sizes(const TestPlan* plans, size_t n) {
  for (size_t t = 0; t < n; ++t)
    if (plans[t].d.n_rowk >= 2147483647)
      return set_error(ETEST_EINVAL, "too many resampling row units");
  for (int s = 0; s < S_COUNT; ++s) {
    int64_t total = 0;
    for (size_t t = 0; t < n; ++t) {
      total += plans[t].wg[s];
      if (total > 2147483647LL || total * slot_threads(s) > 4294967295LL)
        return set_error(ETEST_EINVAL, "launch of slot " + std::to_string(s) + " too large (" +
                                           std::to_string(total) +
                                           "+ workgroups): fewer splits or fewer tests per call");
    }
  }
  return ETEST_OK;
}

// A split stream of more workgroups than the chip holds at once (8 per CU of MI355X's 256)
// keeps every CU's vector ALU busy; there 32 splits per workgroup instead of 16 keep twice as
// many lanes of each selection scan busy, and fewer, larger workgroups leave more room to
// the memory-bound stages beside it (the batched workload of 256 tests: 6.53-6.60 ->
// 6.36-6.37 ms per step).  Smaller streams keep 16: they are latency-bound walks, and
// halving their workgroup count would leave CUs idle.
etest_status build_batch(const etest_request* reqs, int64_t n, bool internal_perm, Batch* b) {
  b->plans.clear();
  b->member_wide = false;
  b->plans.reserve((size_t)n);
  for (int64_t t = 0; t < n; ++t) {
    etest_status s = validate_request(reqs[t]);
    if (s != ETEST_OK) return s;
    TestPlan P = make_plan(reqs[t]);
    if (internal_perm && reqs[t].perm_stats == nullptr && reqs[t].B > 0) {
      P.off[B_PERMOUT] = P.bytes;
      P.size[B_PERMOUT] = (size_t)reqs[t].B * 8;
      P.bytes += align256((size_t)reqs[t].B * 8);
      P.internal_perm = true;
    }
    b->plans.push_back(P);
  }
  // an MMD test fed by an ED test skips its own staging and Gram (and its split stream
  // when it is the same one)
  const Pairing pairing = pair_tests(reqs, n);
  for (int64_t s = 0; s < n; ++s) {
    const int u = pairing.partner[(size_t)s];
    b->plans[(size_t)s].partner = u;
    b->plans[(size_t)s].share_z = pairing.share_z[(size_t)s] != 0;
    if (u < 0) continue;
    for (int k : {S_COLPART, S_COLMEAN, S_STAGE}) b->plans[(size_t)u].wg[k] = 0;
    for (int k : GRAM_SLOTS) b->plans[(size_t)u].wg[k] = 0;
    if (pairing.share_z[(size_t)s]) b->plans[(size_t)u].wg[S_MEMBER] = 0;
  }
  int64_t member_wg = 0;
  for (const TestPlan& P : b->plans) member_wg += P.wg[S_MEMBER];
  if (member_wg > MEMBER_WIDE_MIN_WG) {
    b->member_wide = true;
    for (TestPlan& P : b->plans)
      if (P.wg[S_MEMBER] > 0) P.wg[S_MEMBER] = P.d.B_pad / MEMBER_SPLITS_WIDE;
  }
  return check_launch_sizes(b->plans.data(), b->plans.size());
}

void assign_pointers(TestPlan& P, char* r, DevResult* result) {
  TestDesc& d = P.d;
  d.colpart = (double*)(r + P.off[B_COLPART]);
  d.colmean = (double*)(r + P.off[B_COLMEAN]);
  d.W = r + P.off[B_W];
  d.nrm = r + P.off[B_NRM];
  d.D = r + P.off[B_D];
  d.tsum = (double*)(r + P.off[B_TSUM]);
  d.tmax = (float*)(r + P.off[B_TMAX]);
  d.rsum = (double*)(r + P.off[B_RSUM]);
  d.obs = (double*)(r + P.off[B_OBS]);
  d.planes = r + P.off[B_PLANES];
  d.Z = (uint32_t*)(r + P.off[B_Z]);
  d.part = (double*)(r + P.off[B_PART]);
  d.pstat = (double*)(r + P.off[B_PSTAT]);
  d.flags = (int32_t*)(r + P.off[B_FLAGS]);
  d.result = result;
  // perm_out stays the caller's pointer (possibly NULL: no per-split output) unless an
  // internal output buffer was appended to this test's region
  if (P.internal_perm) d.perm_out = (double*)(r + P.off[B_PERMOUT]);
}

// One device workspace per (device, stream) for the asynchronous entry points.  Calls on
// one stream run in stream order, so each call can reuse the workspace of the previous one
// without waiting for it.  (With a workspace allocated and freed per call, and descriptors
// copied from pageable memory, each call instead waited on the host for the device: 0.5 ms
// of host time per plain_f32 test, the whole step.)  A call that needs more than the
// cached size replaces it with hipFree / hipMalloc, which wait for the device (growth
// only).  The entry's lock is held from placement until the call's pass is enqueued, so
// that two callers on one stream cannot interleave launches over the same memory.  The
// memory stays held until the process ends.
struct StreamWorkspace {
  int dev;
  hipStream_t st;
  std::mutex mu;  // held from placement until the pass is enqueued
  void* ws = nullptr;
  size_t bytes = 0;
};
static std::mutex g_sws_mu;
static std::vector<std::unique_ptr<StreamWorkspace>> g_sws;

static hipError_t stream_workspace(hipStream_t st, size_t total, void** out,
                                   std::unique_lock<std::mutex>* hold) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  StreamWorkspace* c = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_sws_mu);
    for (auto& p : g_sws)
      if (p->dev == dev && p->st == st) c = p.get();
    if (!c) {
      g_sws.push_back(std::make_unique<StreamWorkspace>());
      c = g_sws.back().get();
      c->dev = dev;
      c->st = st;
    }
  }
  std::unique_lock<std::mutex> lk(c->mu);
  if (!c->ws || c->bytes < total) {
    if (c->ws) (void)hipFree(c->ws);  // waits for the device first: rare (growth only)
    c->ws = nullptr;
    c->bytes = 0;
    e = hipMalloc(&c->ws, total);
    if (e != hipSuccess || !c->ws) {
      c->ws = nullptr;
      return e != hipSuccess ? e : hipErrorOutOfMemory;
    }
    c->bytes = total;
  }
  *out = c->ws;
  *hold = std::move(lk);
  return hipSuccess;
}

// Pinned staging for the descriptor tables of asynchronous batches: a small ring per host
// thread.  A slot is handed out again only once the copy from it has run (an event recorded
// after the copy), so a caller can run a few calls ahead of the device.
struct PinnedSlot {
  void* buf = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};
constexpr int PINNED_SLOTS = 4;
static thread_local PinnedSlot g_pinned[PINNED_SLOTS];
static thread_local int g_pinned_next = 0;

static PinnedSlot* pinned_slot(size_t bytes) {
  PinnedSlot& s = g_pinned[g_pinned_next];
  g_pinned_next = (g_pinned_next + 1) % PINNED_SLOTS;
  if (s.used && hipEventSynchronize(s.done) != hipSuccess) return nullptr;
  s.used = false;
  if (s.cap < bytes) {
    if (s.buf) (void)hipHostFree(s.buf);
    s.buf = nullptr;
    s.cap = 0;
    if (hipHostMalloc(&s.buf, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    s.cap = bytes;
  }
  if (!s.done && hipEventCreateWithFlags(&s.done, hipEventDisableSystemFence |
                                                      hipEventDisableTiming) != hipSuccess)
    return nullptr;
  return &s;
}

etest_status place_batch(Batch* b, hipStream_t st, bool stream_ordered) {
  const int n = (int)b->plans.size();
  const size_t desc_bytes = align256(sizeof(TestDesc) * (size_t)n);
  const size_t offs_bytes = align256(sizeof(int64_t) * (size_t)S_COUNT * (size_t)(n + 1));
  const size_t res_bytes = align256(sizeof(DevResult) * (size_t)n);
  size_t total = desc_bytes + offs_bytes + res_bytes;
  std::vector<size_t> base((size_t)n);
  for (int t = 0; t < n; ++t) {
    base[(size_t)t] = total;
    total += b->plans[(size_t)t].bytes;
  }
  void* ws = nullptr;
  hipError_t e = b->cached ? stream_workspace(st, total, &ws, &b->ws_hold)
                 : stream_ordered ? hipMallocAsync(&ws, total, st)
                                  : hipMalloc(&ws, total);
  if (e != hipSuccess || !ws) {
    (void)hipGetLastError();
    return set_error(ETEST_ENOMEM, "device workspace of " + std::to_string(total) + " bytes: " +
                                       hipGetErrorString(e));
  }
  b->ws = ws;
  b->ws_bytes = total;
  b->base = base;
  char* w = (char*)ws;
  b->d_descs = (TestDesc*)w;
  b->d_offs = (int64_t*)(w + desc_bytes);
  b->d_results = (DevResult*)(w + desc_bytes + offs_bytes);
  b->descs.resize((size_t)n);
  b->offs.assign((size_t)S_COUNT * (size_t)(n + 1), 0);
  Pairing pairing;
  pairing.partner.resize((size_t)n);
  pairing.share_z.resize((size_t)n);
  for (int t = 0; t < n; ++t) {
    TestPlan& P = b->plans[(size_t)t];
    assign_pointers(P, w + base[(size_t)t], b->d_results + t);
    b->descs[(size_t)t] = P.d;
    pairing.partner[(size_t)t] = P.partner;
    pairing.share_z[(size_t)t] = P.share_z ? 1 : 0;
    for (int s = 0; s < S_COUNT; ++s)
      b->offs[(size_t)s * (n + 1) + t + 1] = b->offs[(size_t)s * (n + 1) + t] + P.wg[s];
  }
  link_partners(b->descs.data(), pairing);
  for (int t = 0; t < n; ++t) b->plans[(size_t)t].d = b->descs[(size_t)t];
  if (b->desc_by_kernel) {
    // one test: its descriptor and launch table travel as kernel arguments (no host
    // buffer has to outlive the call), and the same kernel clears the flag words
    launch_put_desc(b->descs[0], b->offs.data(), b->d_descs, b->d_offs, st);
    e = hipGetLastError();
  } else if (b->desc_pinned) {
    // descriptors and launch tables are adjacent on the device: one copy of both
    PinnedSlot* slot = pinned_slot(desc_bytes + offs_bytes);
    if (!slot) return set_error(ETEST_ENOMEM, "pinned staging slot");
    char* h = (char*)slot->buf;
    std::memcpy(h, b->descs.data(), sizeof(TestDesc) * (size_t)n);
    std::memcpy(h + desc_bytes, b->offs.data(), sizeof(int64_t) * b->offs.size());
    e = hipMemcpyAsync(b->d_descs, h, desc_bytes + offs_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(slot->done, st);
    slot->used = e == hipSuccess;
  } else {
    e = hipMemcpyAsync(b->d_descs, b->descs.data(), sizeof(TestDesc) * (size_t)n,
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_offs, b->offs.data(), sizeof(int64_t) * b->offs.size(),
                         hipMemcpyHostToDevice, st);
  }
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string("descriptor copy: ") + hipGetErrorString(e));
  return ETEST_OK;
}

void free_batch(Batch* b, hipStream_t st, bool stream_ordered) {
  if (b->ws_hold.owns_lock()) b->ws_hold.unlock();
  if (b->ws && !b->cached) {
    if (stream_ordered) (void)hipFreeAsync(b->ws, st);
    else (void)hipFree(b->ws);
  }
  b->ws = nullptr;
}

// Split stream after the block stage once it has more workgroups than the chip holds at
// once (8 per CU of MI355X's 256), or when the block stage runs on super tiles, whose
// workgroups take a CU's LDS and register file whole and leave the split stream no room
// beside them.  ETEST_SPLIT_LATE = 0 / 1 forces either order.
constexpr int64_t SPLIT_EARLY_MAX_WG = 8 * 256;
static bool split_late(int64_t member_wg, int64_t super_wg) {
  static const int env = env_int("ETEST_SPLIT_LATE", -1, -1, 1);
  if (env >= 0) return env == 1;
  return member_wg > SPLIT_EARLY_MAX_WG || super_wg > 0;
}

void enqueue_stages(const TestDesc* D, const int64_t* d_offs, const int64_t* h_offs, int n,
                    bool dual, hipStream_t st, const uint32_t* import_words, int64_t import_bpad,
                    const StageEvents* ev, const Fork* fork, bool clear_flags,
                    bool member_wide) {
  auto offs = [&](Slot s) { return d_offs + (size_t)s * (n + 1); };
  auto total = [&](Slot s) { return h_offs[(size_t)s * (n + 1) + n]; };
  auto begin = [&](int k, hipStream_t s) {
    if (ev && (ev->mask >> k & 1u)) (void)hipEventRecord(ev->begin[k], s);
  };
  auto end = [&](int k, hipStream_t s) {
    if (ev && (ev->mask >> k & 1u)) (void)hipEventRecord(ev->end[k], s);
  };
  if (clear_flags) launch_clear_flags(st, D, nullptr, n);
  begin(0, st);
  launch_colpart(total(S_COLPART), st, D, offs(S_COLPART), n);
  launch_colmean(total(S_COLMEAN), st, D, offs(S_COLMEAN), n);
  launch_stage(total(S_STAGE), st, D, offs(S_STAGE), n);
  end(0, st);
  // Split stream: independent of the data, so it runs beside other stages.  A stream that
  // fits on the chip at once (up to SPLIT_EARLY_MAX_WG workgroups: each one's walk over the
  // pooled items is latency-bound) is forked after staging, a short memory-bound stage, and
  // runs beside the 128-tile block stage, whose grid leaves room on the CUs.  A larger one
  // (many tests in one launch) keeps every CU's vector ALU busy for its whole duration and
  // would slow the block stage by about as much as it overlaps, and super-tile workgroups
  // leave it no room; then it is forked after the block stage and runs beside the sums and
  // the centring, which are bound by memory.
  hipStream_t ms = st;
  const bool late = fork && split_late(total(S_MEMBER), total(S_GRAM_F32S) + total(S_GRAM_BF16S));
  auto split = [&]() {
    if (fork) {
      (void)hipEventRecord(fork->start, st);
      (void)hipStreamWaitEvent(fork->aux, fork->start, 0);
      ms = fork->aux;
    }
    begin(2, ms);
    if (import_words) launch_member_import(import_bpad, ms, D, import_words);
    else launch_member(total(S_MEMBER), ms, D, offs(S_MEMBER), n, member_wide);
    end(2, ms);
    if (fork) (void)hipEventRecord(fork->done, ms);
  };
  if (!late) split();
  begin(1, st);
  launch_gram_slots(offs, total, st, D, n, dual);
  end(1, st);
  if (late) split();
  begin(3, st);
  launch_rowsum(total(S_ROWSUM), st, D, offs(S_ROWSUM), n);
  launch_observed(st, D, nullptr, n);
  end(3, st);
  begin(4, st);
  launch_center(true, total(S_CENTER_F64), st, D, offs(S_CENTER_F64), n);
  launch_center(false, total(S_CENTER_SPLIT), st, D, offs(S_CENTER_SPLIT), n);
  end(4, st);
  if (fork) (void)hipStreamWaitEvent(st, fork->done, 0);
  begin(5, st);
  launch_perm(0, total(S_PERM_F64), st, D, offs(S_PERM_F64), n, nullptr);
  launch_perm(2, total(S_PERM_S2), st, D, offs(S_PERM_S2), n, nullptr);
  launch_perm(3, total(S_PERM_S3), st, D, offs(S_PERM_S3), n, nullptr);
  end(5, st);
  begin(6, st);
  launch_pstat(total(S_PSTAT), st, D, offs(S_PSTAT), n);
  end(6, st);
}

void enqueue_batch(const Batch& b, hipStream_t st, const uint32_t* import_words,
                   const StageEvents* ev, const Fork* fork) {
  bool dual = false;
  for (const TestPlan& P : b.plans) dual = dual || P.partner >= 0;
  enqueue_stages(b.d_descs, b.d_offs, b.offs.data(), (int)b.plans.size(), dual, st, import_words,
                 import_words ? b.plans[0].d.B_pad : 0, ev, fork, !b.desc_by_kernel,
                 b.member_wide);
}

// Fork/join and stage events only order work on this device (and time it): they skip the
// system-scope fence a default event adds on every record, which costs several
// microseconds per record between the kernels of a pass.
constexpr unsigned kFenceFree = hipEventDisableSystemFence;

// Per-thread auxiliary stream and fork/join events.
static const Fork* thread_fork() {
  static thread_local Fork f;
  static thread_local int state = 0;  // 0 untried, 1 ready, -1 unavailable
  if (state == 0) {
    state = -1;
    if (hipStreamCreateWithFlags(&f.aux, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&f.start, kFenceFree | hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&f.done, kFenceFree | hipEventDisableTiming) == hipSuccess)
      state = 1;
  }
  return state == 1 ? &f : nullptr;
}

// ------------------------------------------------------------------ stage timing
// Each enqueued pass takes its own set of stage events, so passes enqueued back to back
// without a wait in between (the asynchronous entry points) are all timed; the sets are
// read, and returned to the spare list, when the host collects.
struct Profile {
  bool on = false;
  uint32_t mask = 0;
  std::vector<StageEvents*> pending, spare;
  double ms[NSTAGE] = {};
  int64_t launches[NSTAGE] = {};
};
static thread_local Profile g_prof;

static const StageEvents* profile_events() {
  if (!g_prof.on) return nullptr;
  StageEvents* ev = nullptr;
  if (!g_prof.spare.empty()) {
    ev = g_prof.spare.back();
    g_prof.spare.pop_back();
  } else {
    ev = new StageEvents;
    for (int k = 0; k < NSTAGE; ++k)
      if (hipEventCreateWithFlags(&ev->begin[k], kFenceFree) != hipSuccess ||
          hipEventCreateWithFlags(&ev->end[k], kFenceFree) != hipSuccess) {
        delete ev;  // (events created so far are leaked; creation failing means a dead device)
        return nullptr;
      }
  }
  ev->mask = g_prof.mask;
  g_prof.pending.push_back(ev);
  return ev;
}

// Adds the elapsed times of every pending pass (waiting for their last events).
static void profile_collect() {
  for (StageEvents* ev : g_prof.pending) {
    for (int k = 0; k < NSTAGE; ++k) {
      if (!(ev->mask >> k & 1u)) continue;
      float ms = 0.0f;
      if (hipEventSynchronize(ev->end[k]) == hipSuccess &&
          hipEventElapsedTime(&ms, ev->begin[k], ev->end[k]) == hipSuccess) {
        g_prof.ms[k] += ms;
        g_prof.launches[k] += 1;
      } else {
        (void)hipGetLastError();  // a stage this pass did not run (e.g. a cross test's
                                  // resampling): its events were never recorded
      }
    }
    g_prof.spare.push_back(ev);
  }
  g_prof.pending.clear();
}

etest_status dev_to_result(const DevResult& r, etest_result* out) {
  if (r.status == 2) return set_error(ETEST_ENONFINITE, "X or Y contains NaN or Inf");
  if (r.status == 1) return set_error(ETEST_EINVAL, "a supplied split does not hold exactly nx members");
  out->statistic = r.statistic;
  out->threshold = r.threshold;
  out->p_value = r.p_value;
  out->count_ge = r.count_ge;
  out->B = r.B;
  out->n_refined = r.n_refined;
  return ETEST_OK;
}

// Pinned staging for result copies (one per thread).
static DevResult* pinned_results(size_t n) {
  static thread_local DevResult* buf = nullptr;
  static thread_local size_t cap = 0;
  if (cap < n) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    if (hipHostMalloc((void**)&buf, sizeof(DevResult) * n, hipHostMallocDefault) != hipSuccess)
      return nullptr;
    cap = n;
  }
  return buf;
}

void init_pool_once() {
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
}

// Run n tests described by device pointers; waits; fills outs.
static etest_status run_device(const etest_request* reqs, int64_t n, hipStream_t st,
                               etest_result* outs, const uint32_t* import_words = nullptr) {
  init_pool_once();
  Batch b;
  etest_status s = build_batch(reqs, n, false, &b);
  if (s != ETEST_OK) return s;
  s = place_batch(&b, st, true);
  if (s != ETEST_OK) return s;
  enqueue_batch(b, st, import_words, profile_events(), thread_fork());
  hipError_t e = hipGetLastError();
  DevResult* hr = pinned_results((size_t)n);
  if (e == hipSuccess && hr)
    e = hipMemcpyAsync(hr, b.d_results, sizeof(DevResult) * (size_t)n, hipMemcpyDeviceToHost, st);
  free_batch(&b, st, true);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (!hr) return set_error(ETEST_ENOMEM, "pinned result buffer");
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string("run: ") + hipGetErrorString(e));
  profile_collect();
  etest_status worst = ETEST_OK;
  for (int64_t t = 0; t < n; ++t) {
    etest_result tmp;
    etest_status r = dev_to_result(hr[t], &tmp);
    if (r == ETEST_OK) outs[t] = tmp;
    else if (worst == ETEST_OK) worst = r;
  }
  return worst;
}

// Host-buffer path: stage X, Y to the device, run, copy results back.
static etest_status run_host(int kind, int prec, const void* X, int64_t nx, const void* Y,
                             int64_t ny, int64_t p, double gamma, int64_t B, uint64_t seed,
                             double* perm_stats, etest_result* out) {
  if (!out) return set_error(ETEST_EINVAL, "out must not be NULL");
  etest_request r{};
  r.kind = kind;
  r.prec = prec;
  r.nx = nx;
  r.ny = ny;
  r.p = p;
  r.B = B;
  r.seed = seed;
  r.gamma = gamma;
  r.X = X;
  r.Y = Y;
  etest_status s = validate_request(r);
  if (s != ETEST_OK) return s;
  init_pool_once();
  hipStream_t st = nullptr;
  HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
  const size_t el = prec == ETEST_PREC_F64 ? 8 : 4;
  const size_t bx = (size_t)nx * p * el, by = (size_t)ny * p * el;
  void *dx = nullptr, *dy = nullptr;
  double* dp = nullptr;
  hipError_t e = hipMallocAsync(&dx, bx, st);
  if (e == hipSuccess) e = hipMallocAsync(&dy, by, st);
  if (e == hipSuccess && perm_stats && B > 0) e = hipMallocAsync((void**)&dp, (size_t)B * 8, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (dx) (void)hipFreeAsync(dx, st);
    if (dy) (void)hipFreeAsync(dy, st);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    return set_error(ETEST_ENOMEM, "device input buffers");
  }
  e = hipMemcpyAsync(dx, X, bx, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dy, Y, by, hipMemcpyHostToDevice, st);
  r.X = dx;
  r.Y = dy;
  r.perm_stats = dp;
  etest_result res{};
  s = e == hipSuccess ? run_device(&r, 1, st, &res)
                      : set_error(ETEST_EDEVICE, std::string("input copy: ") + hipGetErrorString(e));
  if (s == ETEST_OK && dp) {
    e = hipMemcpyAsync(perm_stats, dp, (size_t)B * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = set_error(ETEST_EDEVICE, std::string("result copy: ") + hipGetErrorString(e));
  }
  (void)hipFreeAsync(dx, st);
  (void)hipFreeAsync(dy, st);
  if (dp) (void)hipFreeAsync(dp, st);
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  if (s == ETEST_OK) *out = res;
  return s;
}

// ------------------------------------------------------------------ graph cache
// Graph replay.  The launch sequence of a list of tests depends only on their shapes
// (nx, ny, p, B, kind, precision) and the tuning rules: every kernel reads its pointers,
// seed and gamma from the descriptor table in device memory.  So a captured graph serves
// any request list of the same shapes: each call rewrites the descriptors (one copy from
// pinned memory) and replays the graph on its own workspace.  Up to kGraphCacheMax graphs
// are kept (least recently used first out), each holding its workspace.
struct ShapeKey {
  int32_t kind, prec;
  int64_t nx, ny, p, B;
  int partner;  // shared block stage (pair_tests), which changes the launch sequence
  int share_z;
  bool operator==(const ShapeKey& o) const {
    return kind == o.kind && prec == o.prec && nx == o.nx && ny == o.ny && p == o.p &&
           B == o.B && partner == o.partner && share_z == o.share_z;
  }
};
static ShapeKey shape_of(const etest_request& r, const Pairing& pg, int64_t t) {
  return ShapeKey{r.kind, r.prec, r.nx, r.ny, r.p, r.B, pg.partner[(size_t)t],
                  (int)pg.share_z[(size_t)t]};
}

struct GraphEntry {
  std::vector<ShapeKey> key;
  uint64_t tune_gen = 0;  // tuning rules the captured work shapes came from
  hipStream_t stream = nullptr;  // calls on one stream share the entry's workspace in order
  Batch batch;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
static std::mutex g_graph_mu;
static std::list<GraphEntry> g_graphs;
static const size_t kGraphCacheMax = 4;

static bool same_shapes(const GraphEntry& g, const etest_request* b, int64_t n, uint64_t gen,
                        const Pairing& pg, hipStream_t st) {
  if (g.stream != st || g.tune_gen != gen || (int64_t)g.key.size() != n) return false;
  for (int64_t t = 0; t < n; ++t)
    if (!(g.key[(size_t)t] == shape_of(b[t], pg, t))) return false;
  return true;
}

static void destroy_entry(GraphEntry& g) {
  // an asynchronous replay of it may still be queued
  (void)hipDeviceSynchronize();
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  free_batch(&g.batch, nullptr, false);
}

static TestDesc* pinned_descs(size_t n) {
  static thread_local TestDesc* buf = nullptr;
  static thread_local size_t cap = 0;
  if (cap < n) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    if (hipHostMalloc((void**)&buf, sizeof(TestDesc) * n, hipHostMallocDefault) != hipSuccess)
      return nullptr;
    cap = n;
  }
  return buf;
}

// The cached graph of a request list on stream st, captured on first use (g_graph_mu held).
static etest_status graph_entry(const etest_request* reqs, int64_t n, hipStream_t st,
                                const Pairing& pairing, GraphEntry** out) {
  const uint64_t gen = tune_generation();
  for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
    if (same_shapes(*it, reqs, n, gen, pairing, st)) {
      g_graphs.splice(g_graphs.begin(), g_graphs, it);
      *out = &g_graphs.front();
      return ETEST_OK;
    }
  GraphEntry g;
  for (int64_t t = 0; t < n; ++t) g.key.push_back(shape_of(reqs[t], pairing, t));
  g.tune_gen = gen;
  g.stream = st;
  etest_status s = build_batch(reqs, n, false, &g.batch);
  if (s != ETEST_OK) return s;
  // Workspace and tables are placed before capture; the graph holds kernels only.
  s = place_batch(&g.batch, st, false);
  if (s != ETEST_OK) {
    free_batch(&g.batch, nullptr, false);
    return s;
  }
  HIP_OK(hipStreamSynchronize(st), "descriptor copy");
  hipStream_t cap = nullptr;
  HIP_OK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    enqueue_batch(g.batch, cap, nullptr, nullptr, thread_fork());
    e = hipStreamEndCapture(cap, &g.graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    destroy_entry(g);
    return set_error(ETEST_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  g_graphs.push_front(std::move(g));
  while (g_graphs.size() > kGraphCacheMax) {
    destroy_entry(g_graphs.back());
    g_graphs.pop_back();
  }
  *out = &g_graphs.front();
  return ETEST_OK;
}

// This call's pointers, seeds and gammas (and, asynchronous calls, result addresses) into
// host descriptors for the entry's tables.
static void fill_descs(const GraphEntry& g, const etest_request* reqs, int64_t n,
                       const Pairing& pairing, TestDesc* hd, etest_result* d_outs) {
  const Batch& b = g.batch;
  for (int64_t t = 0; t < n; ++t) {
    TestPlan P = make_plan(reqs[t]);
    assign_pointers(P, (char*)b.ws + b.base[(size_t)t], b.d_results + t);
    if (d_outs) P.d.out6 = (double*)(d_outs + t);
    hd[t] = P.d;
  }
  link_partners(hd, pairing);
}

static etest_status run_batch_graph(const etest_request* reqs, int64_t n, hipStream_t st,
                                    etest_result* outs) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  const Pairing pairing = pair_tests(reqs, n);
  GraphEntry* hit = nullptr;
  etest_status s = graph_entry(reqs, n, st, pairing, &hit);
  if (s != ETEST_OK) return s;
  Batch& b = hit->batch;
  TestDesc* hd = pinned_descs((size_t)n);
  DevResult* hr = pinned_results((size_t)n);
  if (!hd || !hr) return set_error(ETEST_ENOMEM, "pinned staging buffer");
  fill_descs(*hit, reqs, n, pairing, hd, nullptr);
  HIP_OK(hipMemcpyAsync(b.d_descs, hd, sizeof(TestDesc) * (size_t)n, hipMemcpyHostToDevice, st),
         "descriptor copy");
  HIP_OK(hipGraphLaunch(hit->exec, st), "graph launch");
  HIP_OK(hipMemcpyAsync(hr, b.d_results, sizeof(DevResult) * (size_t)n, hipMemcpyDeviceToHost, st),
         "result copy");
  HIP_OK(hipStreamSynchronize(st), "batch");
  etest_status worst = ETEST_OK;
  for (int64_t t = 0; t < n; ++t) {
    etest_result tmp;
    etest_status r = dev_to_result(hr[t], &tmp);
    if (r == ETEST_OK) outs[t] = tmp;
    else if (worst == ETEST_OK) worst = r;
  }
  return worst;
}

// The graph replay without waiting: descriptors from a pinned staging slot (reused once its
// copy has run), results written into d_outs by each test's last kernel.
static etest_status enqueue_batch_graph(const etest_request* reqs, int64_t n, hipStream_t st,
                                        etest_result* d_outs) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  const Pairing pairing = pair_tests(reqs, n);
  GraphEntry* hit = nullptr;
  etest_status s = graph_entry(reqs, n, st, pairing, &hit);
  if (s != ETEST_OK) return s;
  PinnedSlot* slot = pinned_slot(sizeof(TestDesc) * (size_t)n);
  if (!slot) return set_error(ETEST_ENOMEM, "pinned staging slot");
  fill_descs(*hit, reqs, n, pairing, (TestDesc*)slot->buf, d_outs);
  HIP_OK(hipMemcpyAsync(hit->batch.d_descs, slot->buf, sizeof(TestDesc) * (size_t)n,
                        hipMemcpyHostToDevice, st),
         "descriptor copy");
  HIP_OK(hipEventRecord(slot->done, st), "staging event");
  slot->used = true;
  HIP_OK(hipGraphLaunch(hit->exec, st), "graph launch");
  return ETEST_OK;
}

}  // namespace et

using namespace et;

extern "C" {

const char* etest_last_error(void) { return g_err.c_str(); }

etest_status etest_tune_set(int32_t prec, int64_t n_lo, int64_t n_hi, int32_t kc, int32_t cc) {
  if (prec != ETEST_PREC_F64 && prec != ETEST_PREC_F32 && prec != ETEST_PREC_BF16_REFINED)
    return set_error(ETEST_EINVAL, "unknown precision");
  const int cc_max = prec == ETEST_PREC_F64 ? MAX_CC : 2;
  if (n_lo < 0 || n_hi <= n_lo || kc < 1 || kc > 256 || cc < 1 || cc > cc_max)
    return set_error(ETEST_EINVAL, "bad tuning rule");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.push_back(TuneRule{prec, n_lo, n_hi, kc, cc});
  ++g_tune_gen;
  return ETEST_OK;
}

etest_status etest_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  g_tune_gram.clear();
  ++g_tune_gen;
  return ETEST_OK;
}

etest_status etest_tune_set_gram(int32_t prec, int64_t n_lo, int64_t n_hi, int32_t shape) {
  if (prec != ETEST_PREC_F32 && prec != ETEST_PREC_BF16_REFINED)
    return set_error(ETEST_EINVAL, "Gram shape rules apply to the FP32 and BF16-refined forms");
  if (n_lo < 0 || n_hi <= n_lo || (shape != GSHAPE_TILE && shape != GSHAPE_SUPER))
    return set_error(ETEST_EINVAL, "bad Gram shape rule");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_gram.push_back(GramRule{prec, n_lo, n_hi, shape});
  ++g_tune_gen;
  return ETEST_OK;
}

etest_status etest_profile_enable(int32_t on) {
  if (on < 0) return set_error(ETEST_EINVAL, "profile mask must be >= 0");
  profile_collect();  // passes still pending belong to the previous setting: drop their times
  g_prof.on = on != 0;
  // 1: every stage; any other value: a bit mask of stages shifted left by one
  g_prof.mask = on == 1 ? (1u << NSTAGE) - 1u : ((uint32_t)on >> 1) & ((1u << NSTAGE) - 1u);
  for (int k = 0; k < NSTAGE; ++k) {
    g_prof.ms[k] = 0.0;
    g_prof.launches[k] = 0;
  }
  return ETEST_OK;
}

etest_status etest_profile_read(double* ms, int64_t* launches, int32_t n) {
  if (!ms || !launches || n < 0 || n > NSTAGE) return set_error(ETEST_EINVAL, "bad arguments");
  profile_collect();
  for (int k = 0; k < n; ++k) {
    ms[k] = g_prof.ms[k];
    launches[k] = g_prof.launches[k];
  }
  return ETEST_OK;
}

etest_status etest_validate(const etest_request* req) {
  if (!req) return set_error(ETEST_EINVAL, "request must not be NULL");
  return validate_request(*req);
}

etest_status etest_footprint(const etest_request* req, int64_t* bytes) {
  if (!req || !bytes) return set_error(ETEST_EINVAL, "NULL argument");
  etest_request r = *req;
  // shapes only: pointers need not be valid for a footprint query
  if (!r.X) r.X = (const void*)1;
  if (!r.Y) r.Y = (const void*)1;
  etest_status s = validate_request(r);
  if (s != ETEST_OK) return s;
  *bytes = (int64_t)make_plan(r).bytes + 4096;
  return ETEST_OK;
}

etest_status ed_test(const float* X, int64_t nx, const float* Y, int64_t ny, int64_t p, int64_t B,
                     uint64_t seed, int32_t prec, double* perm_stats, etest_result* out) {
  if (prec != ETEST_PREC_F32 && prec != ETEST_PREC_BF16_REFINED)
    return set_error(ETEST_EINVAL, "ed_test takes ETEST_PREC_F32 or ETEST_PREC_BF16_REFINED");
  return run_host(ETEST_ED, prec, X, nx, Y, ny, p, 0.0, B, seed, perm_stats, out);
}

etest_status mmd_test(const float* X, int64_t nx, const float* Y, int64_t ny, int64_t p,
                      double gamma, int64_t B, uint64_t seed, int32_t prec, double* perm_stats,
                      etest_result* out) {
  if (prec != ETEST_PREC_F32 && prec != ETEST_PREC_BF16_REFINED)
    return set_error(ETEST_EINVAL, "mmd_test takes ETEST_PREC_F32 or ETEST_PREC_BF16_REFINED");
  return run_host(ETEST_MMD, prec, X, nx, Y, ny, p, gamma, B, seed, perm_stats, out);
}

etest_status ed_test_f64(const double* X, int64_t nx, const double* Y, int64_t ny, int64_t p,
                         int64_t B, uint64_t seed, double* perm_stats, etest_result* out) {
  return run_host(ETEST_ED, ETEST_PREC_F64, X, nx, Y, ny, p, 0.0, B, seed, perm_stats, out);
}

etest_status mmd_test_f64(const double* X, int64_t nx, const double* Y, int64_t ny, int64_t p,
                          double gamma, int64_t B, uint64_t seed, double* perm_stats,
                          etest_result* out) {
  return run_host(ETEST_MMD, ETEST_PREC_F64, X, nx, Y, ny, p, gamma, B, seed, perm_stats, out);
}

etest_status etest_run(const etest_request* req, void* stream, etest_result* out) {
  if (!req || !out) return set_error(ETEST_EINVAL, "NULL argument");
  return run_device(req, 1, (hipStream_t)stream, out);
}

static etest_status enqueue_async(const etest_request* req, int kind, etest_result* d_out,
                                  void* stream) {
  if (!req || !d_out) return set_error(ETEST_EINVAL, "NULL argument");
  if (req->kind != kind) return set_error(ETEST_EINVAL, "request kind does not match the call");
  init_pool_once();
  hipStream_t st = (hipStream_t)stream;
  Batch b;
  etest_status s = build_batch(req, 1, false, &b);
  if (s != ETEST_OK) return s;
  // the stream's cached workspace, except under graph capture (a captured graph keeps its
  // own allocation)
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  const hipError_t ce = hipStreamIsCapturing(st, &cap);
  if (ce != hipSuccess) (void)hipGetLastError();
  b.cached = ce == hipSuccess && cap == hipStreamCaptureStatusNone;
  // the descriptor goes up as kernel arguments, and the final kernel writes the result
  // (the leading part of DevResult) into d_out itself: no copies around the pass
  b.desc_by_kernel = true;
  b.plans[0].d.out6 = (double*)d_out;
  s = place_batch(&b, st, true);
  if (s != ETEST_OK) return s;
  enqueue_batch(b, st, nullptr, profile_events(), thread_fork());
  free_batch(&b, st, true);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string("enqueue: ") + hipGetErrorString(e));
  return ETEST_OK;
}

// n tests enqueued on the stream's cached workspace, one launch per stage over all of them,
// without waiting; test t's result goes to d_outs[t] from its last kernel.
static etest_status enqueue_batch_async(const etest_request* reqs, int64_t n,
                                        etest_result* d_outs, void* stream) {
  init_pool_once();
  hipStream_t st = (hipStream_t)stream;
  Batch b;
  etest_status s = build_batch(reqs, n, false, &b);
  if (s != ETEST_OK) return s;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  const hipError_t ce = hipStreamIsCapturing(st, &cap);
  if (ce != hipSuccess) (void)hipGetLastError();
  b.cached = ce == hipSuccess && cap == hipStreamCaptureStatusNone;
  // pinned staging does not suit a captured graph (the slot would be reused under it)
  b.desc_by_kernel = n == 1;
  b.desc_pinned = n > 1 && b.cached;
  for (int64_t t = 0; t < n; ++t) b.plans[(size_t)t].d.out6 = (double*)(d_outs + t);
  s = place_batch(&b, st, true);
  if (s != ETEST_OK) return s;
  enqueue_batch(b, st, nullptr, profile_events(), thread_fork());
  free_batch(&b, st, true);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string("enqueue: ") + hipGetErrorString(e));
  return ETEST_OK;
}

etest_status ed_test_async(const etest_request* req, etest_result* d_out, void* stream) {
  return enqueue_async(req, ETEST_ED, d_out, stream);
}

etest_status mmd_test_async(const etest_request* req, etest_result* d_out, void* stream) {
  return enqueue_async(req, ETEST_MMD, d_out, stream);
}

etest_status etest_batch(const etest_request* reqs, int64_t n, void* stream, etest_result* outs) {
  if (!reqs || !outs || n < 1) return set_error(ETEST_EINVAL, "reqs/outs must be non-NULL, n >= 1");
  for (int64_t t = 0; t < n; ++t) {
    etest_status s = validate_request(reqs[t]);
    if (s != ETEST_OK) return s;
  }
  // With stage timing on, the batch runs eagerly so that the stage events are recorded
  // (events recorded by graph nodes give no elapsed times).
  if (g_prof.on) return run_device(reqs, n, (hipStream_t)stream, outs);
  return run_batch_graph(reqs, n, (hipStream_t)stream, outs);
}

etest_status etest_batch_async(const etest_request* reqs, int64_t n, void* stream,
                               etest_result* d_outs) {
  if (!reqs || !d_outs || n < 1)
    return set_error(ETEST_EINVAL, "reqs/d_outs must be non-NULL, n >= 1");
  for (int64_t t = 0; t < n; ++t) {
    etest_status s = validate_request(reqs[t]);
    if (s != ETEST_OK) return s;
  }
  // With stage timing on (events in graph nodes give no elapsed times) or under stream
  // capture the pass is enqueued eagerly; otherwise the cached graph is replayed.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  const hipError_t ce = hipStreamIsCapturing((hipStream_t)stream, &cap);
  if (ce != hipSuccess) (void)hipGetLastError();
  const bool capturing = ce != hipSuccess || cap != hipStreamCaptureStatusNone;
  // a captured copy would read the call's host tables after they are gone
  if (capturing && n > 1)
    return set_error(ETEST_EINVAL, "etest_batch_async takes one test under stream capture");
  if (g_prof.on || capturing) return enqueue_batch_async(reqs, n, d_outs, stream);
  return enqueue_batch_graph(reqs, n, (hipStream_t)stream, d_outs);
}

etest_status etest_membership(int64_t nx, int64_t ny, uint64_t seed, int64_t b0, int64_t count,
                              uint32_t* words, void* stream) {
  if (nx < 1 || ny < 1 || nx + ny > 2147483647LL) return set_error(ETEST_EINVAL, "bad nx/ny");
  if (b0 < 0 || count < 0 || !words) return set_error(ETEST_EINVAL, "bad range or NULL words");
  hipStream_t st = (hipStream_t)stream;
  launch_member_public(nx, ny, seed, b0, count, words, st);
  HIP_OK(hipGetLastError(), "membership launch");
  HIP_OK(hipStreamSynchronize(st), "membership");
  return ETEST_OK;
}

etest_status etest_blocks(const etest_request* req, void* dxx, void* dyy, void* dxy, void* stream) {
  if (!req || !dxx || !dyy || !dxy) return set_error(ETEST_EINVAL, "NULL argument");
  etest_request r = *req;
  r.B = 0;
  r.perm_stats = nullptr;
  init_pool_once();
  hipStream_t st = (hipStream_t)stream;
  Batch b;
  etest_status s = build_batch(&r, 1, false, &b);
  if (s != ETEST_OK) return s;
  s = place_batch(&b, st, true);
  if (s != ETEST_OK) return s;
  enqueue_batch(b, st);
  int32_t flag = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(&flag, b.descs[0].flags, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && flag == 0) {
    const int64_t elems = r.nx * r.nx + r.ny * r.ny + r.nx * r.ny;
    launch_unpack(r.prec == ETEST_PREC_F64, elems, st, b.d_descs, dxx, dyy, dxy);
    e = hipGetLastError();
  }
  free_batch(&b, st, true);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string("blocks: ") + hipGetErrorString(e));
  if (flag) return set_error(ETEST_ENONFINITE, "X or Y contains NaN or Inf");
  return ETEST_OK;
}

etest_status etest_perm_stats_from_membership(const etest_request* req, const uint32_t* words,
                                              int64_t count, double* stats, void* stream,
                                              etest_result* out) {
  if (!req || !words || !stats || !out || count < 1)
    return set_error(ETEST_EINVAL, "NULL argument or count < 1");
  etest_request r = *req;
  r.B = count;
  r.perm_stats = stats;
  return run_device(&r, 1, (hipStream_t)stream, out, words);
}

}  // extern "C"

// ------------------------------------------------------------------ cross tests
// One cross test: staging of [x1; y1 | x2; y2], the rectangle of cross tiles with per-row
// sums split by column class, then the statistic (k_cross.hip).  Synchronous.
etest_status etest_cross(const etest_request* req, void* stream, etest_cross_result* out) {
  if (!req || !out) return set_error(ETEST_EINVAL, "NULL argument");
  etest_request r = *req;
  r.B = 0;
  r.perm_stats = nullptr;
  etest_status s = validate_request(r);
  if (s != ETEST_OK) return s;
  if (r.nx < 2 || r.ny < 2) return set_error(ETEST_EINVAL, "cross tests need nx, ny >= 2");
  init_pool_once();
  hipStream_t st = (hipStream_t)stream;
  const int64_t nx1 = r.nx / 2, ny1 = r.ny / 2, nx2 = r.nx - nx1;
  TestDesc d{};
  d.kind = r.kind;
  d.prec = r.prec;
  d.cross = 1;
  d.cnx1 = (int32_t)nx1;
  d.cny1 = (int32_t)ny1;
  d.cnx2 = (int32_t)nx2;
  d.nx = (int32_t)(nx1 + ny1);              // x side
  d.ny = (int32_t)(r.nx + r.ny - nx1 - ny1);  // y side
  d.p = (int32_t)r.p;
  const bool f64 = r.prec == ETEST_PREC_F64;
  d.gop = gram_operands(r.prec, r.p);
  const int kq = gram_k_slice(d.gop);
  d.p_pad = (int32_t)((r.p + kq - 1) / kq * kq);
  d.tx = (d.nx + TILE - 1) / TILE;
  d.ty = (d.ny + TILE - 1) / TILE;
  d.nt = d.tx + d.ty;
  d.ntiles = d.tx * d.ty;
  // cross tests store no block tile, which the super-tile kernel stages its raw Gram
  // entries through: they keep one 128-tile workgroup per tile
  d.gshape = GSHAPE_TILE;
  const int64_t gram_wg = d.ntiles;
  d.refine = f64 ? 0 : 1;
  d.nrowchunks = (int32_t)((r.nx + r.ny + COLSUM_ROWS - 1) / COLSUM_ROWS);
  d.gamma = r.kind == ETEST_MMD ? r.gamma : 0.0;
  d.X = r.X;
  d.Y = r.Y;
  const int64_t npad = (int64_t)d.nt * TILE;
  const size_t el_w = (size_t)gram_operand_bytes(d.gop);
  // workspace: descriptor, launch tables, then the buffers the stages index
  enum { C_DESC, C_OFFS, C_COLPART, C_COLMEAN, C_W, C_NRM, C_TSUM, C_TMAX, C_V, C_OBS, C_FLAGS, C_N };
  size_t sz[C_N];
  sz[C_DESC] = sizeof(TestDesc);
  sz[C_OFFS] = 5 * 2 * sizeof(int64_t);
  sz[C_COLPART] = f64 ? 0 : (size_t)d.nrowchunks * r.p * 8;
  sz[C_COLMEAN] = f64 ? 0 : (size_t)r.p * 8;
  sz[C_W] = (size_t)npad * d.p_pad * el_w;
  sz[C_NRM] = (size_t)npad * (f64 ? 8 : 4);
  sz[C_TSUM] = (size_t)d.ntiles * TSUM_STRIDE * 8;
  sz[C_TMAX] = (size_t)d.ntiles * TMAX_PER_TILE * 4;
  sz[C_V] = (size_t)npad * 8;
  sz[C_OBS] = 8 * 8;
  sz[C_FLAGS] = FLAG_WORDS * 4;
  size_t off[C_N], total = 0;
  for (int k = 0; k < C_N; ++k) {
    off[k] = total;
    total += align256(sz[k]);
  }
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, total, st);
  if (e != hipSuccess || !ws) {
    (void)hipGetLastError();
    return set_error(ETEST_ENOMEM, "cross test workspace of " + std::to_string(total) + " bytes");
  }
  char* w = (char*)ws;
  d.colpart = (double*)(w + off[C_COLPART]);
  d.colmean = (double*)(w + off[C_COLMEAN]);
  d.W = w + off[C_W];
  d.nrm = w + off[C_NRM];
  d.tsum = (double*)(w + off[C_TSUM]);
  d.tmax = (float*)(w + off[C_TMAX]);
  d.rsum = (double*)(w + off[C_V]);
  d.obs = (double*)(w + off[C_OBS]);
  d.flags = (int32_t*)(w + off[C_FLAGS]);
  // launch tables [0, workgroups] of the stages (a one-test batch)
  const bool f32like = !f64;
  const int64_t wg[5] = {f32like ? colpart_wgs(d.nrowchunks, r.p) : 0,
                         f32like ? (r.p + 63) / 64 : 0, stage_wgs(npad, d.p_pad), gram_wg, 0};
  int64_t hoffs[10];
  for (int k = 0; k < 5; ++k) {
    hoffs[2 * k] = 0;
    hoffs[2 * k + 1] = wg[k];
  }
  const TestDesc* D = (const TestDesc*)(w + off[C_DESC]);
  const int64_t* O = (const int64_t*)(w + off[C_OFFS]);
  e = hipMemcpyAsync(w + off[C_DESC], &d, sizeof(TestDesc), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w + off[C_OFFS], hoffs, sizeof(hoffs), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    // stage timing as for the permutation tests: 0 staging, 1 blocks, 6 statistic
    const StageEvents* ev = profile_events();
    auto mark = [&](int k, bool begin) {
      if (ev && (ev->mask >> k & 1u)) (void)hipEventRecord(begin ? ev->begin[k] : ev->end[k], st);
    };
    launch_clear_flags(st, D, nullptr, 1);
    mark(0, true);
    launch_colpart(wg[0], st, D, O, 1);
    launch_colmean(wg[1], st, D, O + 2, 1);
    launch_stage(wg[2], st, D, O + 4, 1);
    mark(0, false);
    mark(1, true);
    launch_gram(d.gop, false, wg[3], st, D, O + 6, 1, false);  // 128-tile shape
    mark(1, false);
    mark(6, true);
    launch_cross_final(st, D);
    mark(6, false);
    e = hipGetLastError();
  }
  // obs[0..3] and flags[0..1] back to the host
  struct Back { double obs[4]; int32_t flags[2]; };
  static thread_local Back* hb = nullptr;
  if (!hb && hipHostMalloc((void**)&hb, sizeof(Back), hipHostMallocDefault) != hipSuccess) hb = nullptr;
  if (e == hipSuccess && hb) e = hipMemcpyAsync(hb->obs, d.obs, 4 * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && hb) e = hipMemcpyAsync(hb->flags, d.flags, 2 * 4, hipMemcpyDeviceToHost, st);
  (void)hipFreeAsync(ws, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (!hb) return set_error(ETEST_ENOMEM, "pinned result buffer");
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string("cross: ") + hipGetErrorString(e));
  profile_collect();
  if (hb->flags[0]) return set_error(ETEST_ENONFINITE, "X or Y contains NaN or Inf");
  out->statistic = hb->obs[0];
  out->sigma = hb->obs[1];
  out->z = hb->obs[2];
  out->p_value = hb->obs[3];
  out->n_refined = hb->flags[1];
  return ETEST_OK;
}

// ------------------------------------------------- baselines: standard and pre-computation
namespace et {

// Staging, blocks, block sums and observed statistic of the first m tests of a batch (the
// launch tables of a prefix of the tests are prefixes of the batch's tables).
static void enqueue_blocks(const Batch& b, int m, hipStream_t st) {
  const int n = (int)b.plans.size();
  auto offs = [&](Slot s) { return b.d_offs + (size_t)s * (n + 1); };
  auto total = [&](Slot s) { return b.offs[(size_t)s * (n + 1) + m]; };
  const TestDesc* D = b.d_descs;
  launch_clear_flags(st, D, nullptr, m);
  launch_colpart(total(S_COLPART), st, D, offs(S_COLPART), m);
  launch_colmean(total(S_COLMEAN), st, D, offs(S_COLMEAN), m);
  launch_stage(total(S_STAGE), st, D, offs(S_STAGE), m);
  launch_gram_slots(offs, total, st, D, m, false);
  launch_rowsum(total(S_ROWSUM), st, D, offs(S_ROWSUM), m);
  launch_observed(st, D, nullptr, m);
}

// Device result -> host, free the workspaces, wait.
static etest_status finish_baseline(DevResult* d_res, Batch* b, void* aux, hipStream_t st,
                                    hipError_t e, const char* what, etest_result* out) {
  DevResult* h = pinned_results(1);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess && h) e = hipMemcpyAsync(h, d_res, sizeof(DevResult), hipMemcpyDeviceToHost, st);
  free_batch(b, st, true);
  if (aux) (void)hipFreeAsync(aux, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (!h) return set_error(ETEST_ENOMEM, "pinned result buffer");
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return dev_to_result(*h, out);
}

// Standard test: the B + 1 splits (drawn splits 0..B-1, identity B) are recomputed in
// passes of up to 256 tests that share one batch workspace; each test stages its split's
// X*, Y* through a row map and runs staging, Gram, block sums and the observed statistic.
static etest_status run_standard(const etest_request& r, hipStream_t st, etest_result* out) {
  init_pool_once();
  const int64_t n = r.nx + r.ny, W = (n + 31) / 32, B = r.B;
  etest_request q = r;
  q.B = 0;
  q.perm_stats = nullptr;
  const TestPlan P0 = make_plan(q, 0, PLAN_BLOCKS);
  const int64_t budget = 4LL << 30;
  const int64_t chunk =
      std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(B + 1, 256),
                                             budget / std::max<int64_t>(1, (int64_t)P0.bytes)));
  size_t aoff[5], asz[5] = {(size_t)(chunk * n * 4), (size_t)(chunk * W * 4),
                            (size_t)((B + 1) * 8), (size_t)(FLAG_WORDS * 4), sizeof(DevResult)};
  size_t atotal = 0;
  for (int k = 0; k < 5; ++k) {
    aoff[k] = atotal;
    atotal += align256(asz[k]);
  }
  void* aux = nullptr;
  hipError_t e = hipMallocAsync(&aux, atotal, st);
  if (e != hipSuccess || !aux) {
    (void)hipGetLastError();
    return set_error(ETEST_ENOMEM, "standard test buffers of " + std::to_string(atotal) + " bytes");
  }
  char* a = (char*)aux;
  int32_t* rowmaps = (int32_t*)(a + aoff[0]);
  uint32_t* words = (uint32_t*)(a + aoff[1]);
  double* stats = (double*)(a + aoff[2]);
  int32_t* flags = (int32_t*)(a + aoff[3]);
  DevResult* d_res = (DevResult*)(a + aoff[4]);
  Batch b;
  b.plans.assign((size_t)chunk, P0);
  for (int64_t k = 0; k < chunk; ++k) b.plans[(size_t)k].d.rowmap = rowmaps + k * n;
  etest_status s = place_batch(&b, st, true);
  if (s != ETEST_OK) {
    (void)hipFreeAsync(aux, st);
    return s;
  }
  e = hipMemsetAsync(flags, 0, FLAG_WORDS * 4, st);
  for (int64_t c0 = 0; e == hipSuccess && c0 <= B; c0 += chunk) {
    const int m = (int)std::min<int64_t>(chunk, B + 1 - c0);
    const int64_t drawn = std::max<int64_t>(0, std::min<int64_t>(m, B - c0));
    launch_member_public(r.nx, r.ny, r.seed, c0, drawn, words, st);
    launch_rowmap(words, drawn, m, n, r.nx, rowmaps, st);
    enqueue_blocks(b, m, st);
    launch_collect(b.d_descs, m, c0, B, stats, flags, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) launch_count(stats, B, flags, r.perm_stats, d_res, st);
  return finish_baseline(d_res, &b, aux, st, e, "standard test", out);
}

// Pre-computation test: the pooled Gram (D_WW: upper tiles, or with `dense` the whole
// nt x nt grid as Alg. 5 prints it), the split stream, then the per-split class sums of
// every stored entry and the statistics.
// Stage timing (etest_profile_enable): 0 staging, 1 blocks, 2 split stream, 5 class sums,
// 6 statistics + p-value.
static etest_status run_precomputed(const etest_request& r, hipStream_t st, etest_result* out,
                                    bool dense) {
  init_pool_once();
  Batch b;
  b.plans.push_back(make_plan(r, 0, dense ? PLAN_PRECOMP_DENSE : PLAN_PRECOMP));
  // one workgroup per (stored tile, 32-row strip, 64 split columns)
  const int64_t groups = (r.B + 1 + 63) / 64;
  if ((int64_t)b.plans[0].d.ntiles * PC_STRIPS > 2147483647LL / groups)
    return set_error(ETEST_EINVAL, "pre-computation test: tiles x strips x split groups must "
                                   "stay below 2^31");
  etest_status s = place_batch(&b, st, true);
  if (s != ETEST_OK) return s;
  const TestDesc& d = b.descs[0];
  const TestDesc* D = b.d_descs;
  auto offs = [&](Slot k) { return b.d_offs + (size_t)k * 2; };
  auto total = [&](Slot k) { return b.offs[(size_t)k * 2 + 1]; };
  const StageEvents* ev = profile_events();
  auto mark = [&](int k, bool begin) {
    if (ev && (ev->mask >> k & 1u)) (void)hipEventRecord(begin ? ev->begin[k] : ev->end[k], st);
  };
  launch_clear_flags(st, D, nullptr, 1);
  mark(0, true);
  launch_colpart(total(S_COLPART), st, D, offs(S_COLPART), 1);
  launch_colmean(total(S_COLMEAN), st, D, offs(S_COLMEAN), 1);
  launch_stage(total(S_STAGE), st, D, offs(S_STAGE), 1);
  mark(0, false);
  mark(2, true);
  launch_member(total(S_MEMBER), st, D, offs(S_MEMBER), 1);
  mark(2, false);
  mark(1, true);
  launch_gram_slots(offs, total, st, D, 1, false);
  mark(1, false);
  mark(5, true);
  launch_precomp(r.prec == ETEST_PREC_F64, D, d.ntiles, r.B, d.part, st);
  mark(5, false);
  mark(6, true);
  launch_precomp_stat(D, d.ntiles, r.B, d.part, d.pstat, st);
  launch_count(d.pstat, r.B, d.flags, r.perm_stats, b.d_results, st);
  mark(6, false);
  etest_status rs = finish_baseline(b.d_results, &b, nullptr, st, hipSuccess, "pre-computation test", out);
  profile_collect();
  return rs;
}

// HSIC independence test: the Gaussian kernel matrices of x and of y as two one-sample Grams
// in one batch (staging and blocks only), then dense zero-diagonal copies, row sums, the
// permutations, the per-permutation terms, the statistics and the p-value.
// Stage timing (etest_profile_enable): 0 staging, 1 blocks, 2 permutations, 3 dense
// matrices and row sums, 5 per-permutation terms, 6 statistics + p-value.
static etest_status run_hsic(const etest_hsic_request& h, hipStream_t st, etest_result* out) {
  init_pool_once();
  const int64_t n = h.n, B = h.B, nperm = h.B + 1;
  const bool f64 = h.prec == ETEST_PREC_F64;
  etest_request rx{}, ry{};
  rx.kind = ry.kind = ETEST_MMD;
  rx.prec = ry.prec = h.prec;
  rx.nx = ry.nx = n;
  rx.ny = ry.ny = 0;  // one sample: the Gram covers the x (or y) rows alone
  rx.p = h.p;
  ry.p = h.q;
  rx.gamma = h.gamma_x;
  ry.gamma = h.gamma_y;
  rx.X = rx.Y = h.X;
  ry.X = ry.Y = h.Y;
  Batch b;
  b.plans.push_back(make_plan(rx, 0, PLAN_BLOCKS));
  b.plans.push_back(make_plan(ry, 0, PLAN_BLOCKS));
  const int64_t nblk = (n + HSIC_RB - 1) / HSIC_RB;
  const size_t el = f64 ? 8 : 4;
  enum { H_KX, H_KY, H_RX, H_RY, H_HS, H_FLAGS, H_PERMS, H_PART, H_STATS, H_RES, H_N };
  size_t sz[H_N] = {(size_t)(n * n) * el, (size_t)(n * n) * el, (size_t)n * 8, (size_t)n * 8,
                    2 * 8, FLAG_WORDS * 4, (size_t)(nperm * n) * 4, (size_t)(nperm * nblk) * 16,
                    (size_t)nperm * 8, sizeof(DevResult)};
  size_t off[H_N], total = 0;
  for (int k = 0; k < H_N; ++k) {
    off[k] = total;
    total += align256(sz[k]);
  }
  void* aux = nullptr;
  hipError_t e = hipMallocAsync(&aux, total, st);
  if (e != hipSuccess || !aux) {
    (void)hipGetLastError();
    return set_error(ETEST_ENOMEM, "HSIC test buffers of " + std::to_string(total) + " bytes");
  }
  char* a = (char*)aux;
  etest_status s = place_batch(&b, st, true);
  if (s != ETEST_OK) {
    (void)hipFreeAsync(aux, st);
    return s;
  }
  double* rxs = (double*)(a + off[H_RX]);
  double* rys = (double*)(a + off[H_RY]);
  double* hs = (double*)(a + off[H_HS]);
  int32_t* flags = (int32_t*)(a + off[H_FLAGS]);
  int32_t* perms = (int32_t*)(a + off[H_PERMS]);
  double* part = (double*)(a + off[H_PART]);
  double* stats = (double*)(a + off[H_STATS]);
  DevResult* d_res = (DevResult*)(a + off[H_RES]);
  const TestDesc* D = b.d_descs;
  auto offs = [&](Slot k) { return b.d_offs + (size_t)k * 3; };
  auto tot = [&](Slot k) { return b.offs[(size_t)k * 3 + 2]; };
  const StageEvents* ev = profile_events();
  auto mark = [&](int k, bool begin) {
    if (ev && (ev->mask >> k & 1u)) (void)hipEventRecord(begin ? ev->begin[k] : ev->end[k], st);
  };
  launch_clear_flags(st, D, nullptr, 2);
  mark(0, true);
  launch_colpart(tot(S_COLPART), st, D, offs(S_COLPART), 2);
  launch_colmean(tot(S_COLMEAN), st, D, offs(S_COLMEAN), 2);
  launch_stage(tot(S_STAGE), st, D, offs(S_STAGE), 2);
  mark(0, false);
  mark(1, true);
  launch_gram_slots(offs, tot, st, D, 2, false);
  mark(1, false);
  mark(2, true);
  launch_permgen(n, h.seed, 0, B, nperm, perms, st);
  mark(2, false);
  mark(3, true);
  launch_hsic_prep(f64, D, n, a + off[H_KX], a + off[H_KY], rxs, rys, hs, flags, st);
  mark(3, false);
  mark(5, true);
  launch_hsic_terms(f64, a + off[H_KX], a + off[H_KY], n, perms, nperm, rxs, rys, part, st);
  mark(5, false);
  mark(6, true);
  launch_hsic_stat(part, n, nperm, hs, stats, st);
  launch_count(stats, B, flags, h.perm_stats, d_res, st);
  mark(6, false);
  etest_status rs = finish_baseline(d_res, &b, aux, st, hipSuccess, "HSIC test", out);
  profile_collect();
  return rs;
}

static etest_status validate_hsic(const etest_hsic_request& h) {
  // The unbiased HSIC is a small difference of three large terms (on high-dimensional data
  // about 1e-5 of the kernel entries under independence): 8-bit coordinates cannot carry it,
  // so the test has the FP64 and FP32 forms only.
  if (h.prec != ETEST_PREC_F64 && h.prec != ETEST_PREC_F32)
    return set_error(ETEST_EINVAL, "HSIC test: prec must be ETEST_PREC_F64 or ETEST_PREC_F32");
  if (h.n < 4 || h.n > HSIC_NMAX)
    return set_error(ETEST_EINVAL, "HSIC test needs 4 <= n <= " + std::to_string(HSIC_NMAX));
  if (h.p < 1 || h.q < 1 || h.p > 2147483647LL || h.q > 2147483647LL)
    return set_error(ETEST_EINVAL, "p and q must be >= 1");
  if (h.B < 0 || h.B >= 2147483647LL) return set_error(ETEST_EINVAL, "B out of range");
  if (!(h.gamma_x > 0.0) || !(h.gamma_y > 0.0) || !std::isfinite(h.gamma_x) ||
      !std::isfinite(h.gamma_y))
    return set_error(ETEST_EINVAL, "gamma_x and gamma_y must be finite and > 0");
  if (!h.X || !h.Y) return set_error(ETEST_EINVAL, "X and Y must not be NULL");
  if (h.reserved != 0) return set_error(ETEST_EINVAL, "reserved field must be 0");
  // the term pass launches one workgroup per (permutation, block of HSIC_RB rows)
  const int64_t nblk = (h.n + HSIC_RB - 1) / HSIC_RB;
  if ((h.B + 1) > 2147483647LL / nblk)
    return set_error(ETEST_EINVAL, "HSIC test: (B + 1) * ceil(n / " + std::to_string(HSIC_RB) +
                                       ") must stay below 2^31");
  return ETEST_OK;
}

}  // namespace et

extern "C" {

etest_status etest_hsic(const etest_hsic_request* req, void* stream, etest_result* out) {
  if (!req || !out) return set_error(ETEST_EINVAL, "NULL argument");
  etest_status s = validate_hsic(*req);
  if (s != ETEST_OK) return s;
  return run_hsic(*req, (hipStream_t)stream, out);
}

etest_status etest_permutations(int64_t n, uint64_t seed, int64_t b0, int64_t count,
                                int32_t* perms, void* stream) {
  if (n < 1 || n > HSIC_NMAX) return set_error(ETEST_EINVAL, "permutations need 1 <= n <= " + std::to_string(HSIC_NMAX));
  if (b0 < 0 || count < 0 || !perms) return set_error(ETEST_EINVAL, "bad range or NULL perms");
  hipStream_t st = (hipStream_t)stream;
  launch_permgen(n, seed, b0, count, count, perms, st);
  HIP_OK(hipGetLastError(), "permutations launch");
  HIP_OK(hipStreamSynchronize(st), "permutations");
  return ETEST_OK;
}

etest_status etest_standard(const etest_request* req, void* stream, etest_result* out) {
  if (!req || !out) return set_error(ETEST_EINVAL, "NULL argument");
  etest_status s = validate_request(*req);
  if (s != ETEST_OK) return s;
  return run_standard(*req, (hipStream_t)stream, out);
}

etest_status etest_precomputed(const etest_request* req, void* stream, etest_result* out) {
  if (!req || !out) return set_error(ETEST_EINVAL, "NULL argument");
  etest_status s = validate_request(*req);
  if (s != ETEST_OK) return s;
  return run_precomputed(*req, (hipStream_t)stream, out, false);
}

etest_status etest_precomputed_dense(const etest_request* req, void* stream, etest_result* out) {
  if (!req || !out) return set_error(ETEST_EINVAL, "NULL argument");
  etest_status s = validate_request(*req);
  if (s != ETEST_OK) return s;
  return run_precomputed(*req, (hipStream_t)stream, out, true);
}

}  // extern "C"
