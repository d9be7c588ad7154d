// Host-only check of the workspace planner: for many request shapes, every buffer of a
// test lies inside its region, buffers do not overlap, sizes cover what the kernels index,
// and the per-split output pointer is the caller's (NULL stays NULL) unless an internal
// buffer was requested.  Kernel launchers are stubbed out: nothing touches a device.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "runtime.h"

namespace et {
void launch_clear_flags(hipStream_t, const TestDesc*, const int64_t*, int) {}
void launch_colpart(int64_t, hipStream_t, const TestDesc*, const int64_t*, int) {}
void launch_colmean(int64_t, hipStream_t, const TestDesc*, const int64_t*, int) {}
void launch_stage(int64_t, hipStream_t, const TestDesc*, const int64_t*, int) {}
void launch_gram(int, bool, int64_t, hipStream_t, const TestDesc*, const int64_t*, int, bool) {}
void launch_gram_finish(int64_t, hipStream_t, const TestDesc*, const int64_t*, int, bool) {}
void launch_rowsum(int64_t, hipStream_t, const TestDesc*, const int64_t*, int) {}
void launch_observed(hipStream_t, const TestDesc*, const int64_t*, int) {}
void launch_center(bool, int64_t, hipStream_t, const TestDesc*, const int64_t*, int) {}
void launch_member(int64_t, hipStream_t, const TestDesc*, const int64_t*, int, bool) {}
void launch_member_public(int64_t, int64_t, uint64_t, int64_t, int64_t, uint32_t*, hipStream_t) {}
void launch_member_import(int64_t, hipStream_t, const TestDesc*, const uint32_t*) {}
void launch_perm(int, int64_t, hipStream_t, const TestDesc*, const int64_t*, int, const int32_t*) {}
void launch_pstat(int64_t, hipStream_t, const TestDesc*, const int64_t*, int) {}
void launch_cross_final(hipStream_t, const TestDesc*) {}
void launch_unpack(bool, int64_t, hipStream_t, const TestDesc*, void*, void*, void*) {}
void launch_rowmap(const uint32_t*, int64_t, int64_t, int64_t, int64_t, int32_t*, hipStream_t) {}
void launch_collect(const TestDesc*, int, int64_t, int64_t, double*, int32_t*, hipStream_t) {}
void launch_count(const double*, int64_t, const int32_t*, double*, DevResult*, hipStream_t) {}
void launch_precomp(bool, const TestDesc*, int64_t, int64_t, double*, hipStream_t) {}
void launch_precomp_stat(const TestDesc*, int64_t, int64_t, const double*, double*, hipStream_t) {}
void launch_permgen(int64_t, uint64_t, int64_t, int64_t, int64_t, int32_t*, hipStream_t) {}
void launch_hsic_prep(bool, const TestDesc*, int64_t, void*, void*, double*, double*, double*,
                      int32_t*, hipStream_t) {}
void launch_hsic_terms(bool, const void*, const void*, int64_t, const int32_t*, int64_t,
                       const double*, const double*, double*, hipStream_t) {}
void launch_hsic_stat(const double*, int64_t, int64_t, const double*, double*, hipStream_t) {}
void launch_put_desc(const TestDesc&, const int64_t*, TestDesc*, int64_t*, hipStream_t) {}
}  // namespace et

using namespace et;

static int failures = 0;
#define CHECK(c, ...)                        \
  do {                                       \
    if (!(c)) {                              \
      std::printf("FAIL %s: ", #c);          \
      std::printf(__VA_ARGS__);              \
      std::printf("\n");                     \
      ++failures;                            \
    }                                        \
  } while (0)

static void check_plan(const etest_request& r, bool internal) {
  Batch b;
  etest_status s = build_batch(&r, 1, internal, &b);
  CHECK(s == ETEST_OK, "build_batch %d", (int)s);
  if (s != ETEST_OK) return;
  TestPlan P = b.plans[0];
  const TestDesc& d0 = P.d;
  const int64_t npad = (int64_t)d0.nt * TILE;
  // what the kernels index, in bytes
  const bool f64 = r.prec == ETEST_PREC_F64;
  size_t need[B_NBUF] = {};
  need[B_W] = (size_t)npad * d0.p_pad * gram_operand_bytes(d0.gop);
  need[B_D] = (size_t)d0.ntiles * TILE * TILE * (f64 ? 8 : 4);
  need[B_PLANES] = (size_t)d0.ntiles * TILE * TILE * (f64 ? 8 : plane_bytes_per_entry(d0.pfmt));
  need[B_Z] = (size_t)d0.nt * TILE_WORDS * d0.B_pad * 4;
  need[B_PART] = (size_t)d0.n_rowk * d0.B_pad * 8;
  need[B_PSTAT] = (size_t)d0.B_pad * 8;
  need[B_RSUM] = (size_t)npad * 16;
  need[B_TSUM] = (size_t)d0.ntiles * 2 * TILE * 8;
  for (int k = 0; k < B_NBUF; ++k) {
    if (k == B_PERMOUT && !P.internal_perm) continue;
    CHECK(P.size[k] >= need[k], "buffer %d: %zu < %zu", k, P.size[k], need[k]);
    CHECK(P.off[k] + P.size[k] <= P.bytes, "buffer %d ends at %zu past %zu", k,
          P.off[k] + P.size[k], P.bytes);
    for (int m = 0; m < k; ++m) {
      if (m == B_PERMOUT && !P.internal_perm) continue;
      if (P.size[k] == 0 || P.size[m] == 0) continue;
      const bool apart = P.off[k] + P.size[k] <= P.off[m] || P.off[m] + P.size[m] <= P.off[k];
      CHECK(apart, "buffers %d and %d overlap", k, m);
    }
  }
  CHECK(d0.B_pad % NP == 0 && d0.B_pad >= d0.B + 1, "B_pad %lld", (long long)d0.B_pad);
  {
    // exactly one Gram slot, matching the test's operand format and workgroup shape (the
    // super-tile Gram with its finish pass, one workgroup per stored tile)
    int used = 0;
    for (int k : GRAM_SLOTS) used += P.wg[k] > 0 ? 1 : 0;
    CHECK(used == (d0.gshape == GSHAPE_SUPER ? 2 : 1), "%d Gram slots used", used);
    const int64_t st = (d0.nt + 1) / 2;
    if (d0.gshape == GSHAPE_SUPER) {
      CHECK(P.wg[d0.gop == GOP_F16PAIR ? S_GRAM_F32S : S_GRAM_BF16S] == st * (st + 1) / 2,
            "super-tile Gram grid");
      CHECK(P.wg[S_GRAM_FIN] == d0.ntiles, "super-tile finish grid");
    } else
      CHECK(P.wg[d0.gop == GOP_F64 ? S_GRAM_F64 : d0.gop == GOP_F16PAIR ? S_GRAM_F32 : S_GRAM_BF16]
                == d0.ntiles, "block-tile Gram grid");
    CHECK(d0.gshape == GSHAPE_TILE || d0.gop != GOP_F64, "FP64 blocks on super tiles");
  }
  CHECK(d0.cc >= 1 && d0.cc <= MAX_CC, "cc %d", d0.cc);
  // pointer assignment inside a fake region (pure address arithmetic, never dereferenced)
  char* base = (char*)(uintptr_t)0x10000000000ull;
  DevResult res;
  assign_pointers(P, base, &res);
  if (P.internal_perm) {
    CHECK((char*)P.d.perm_out >= base && (char*)P.d.perm_out + r.B * 8 <= base + P.bytes,
          "internal perm_out outside the region");
  } else {
    CHECK(P.d.perm_out == r.perm_stats, "perm_out changed from the caller's pointer");
  }
  CHECK((char*)P.d.Z >= base && (char*)P.d.Z + need[B_Z] <= base + P.bytes, "Z outside");
  CHECK((char*)P.d.part >= base && (char*)P.d.part + need[B_PART] <= base + P.bytes,
        "part outside");
}

// Plans of the two baselines: blocks only (one recomputation of the standard test) and the
// pre-computation test (pooled blocks, split stream, strip sums, split statistics).
static void check_mode_plan(const etest_request& r, int mode) {
  const TestPlan P = make_plan(r, 0, mode);
  const TestDesc& d0 = P.d;
  const int64_t npad = (int64_t)d0.nt * TILE;
  const bool f64 = r.prec == ETEST_PREC_F64;
  size_t need[B_NBUF] = {};
  need[B_W] = (size_t)npad * d0.p_pad * gram_operand_bytes(d0.gop);
  need[B_D] = (size_t)d0.ntiles * TILE * TILE * (f64 ? 8 : 4);
  need[B_RSUM] = (size_t)npad * 16;
  need[B_TSUM] = (size_t)d0.ntiles * 2 * TILE * 8;
  const bool precomp = mode == PLAN_PRECOMP || mode == PLAN_PRECOMP_DENSE;
  // the dense pooled matrix: every tile of the nt x nt grid, one 128-tile Gram workgroup each
  const int64_t tiles = mode == PLAN_PRECOMP_DENSE ? (int64_t)d0.nt * d0.nt
                                                   : (int64_t)d0.nt * (d0.nt + 1) / 2;
  CHECK(d0.ntiles == tiles && d0.dense == (mode == PLAN_PRECOMP_DENSE ? 1 : 0),
        "mode %d tile count %d", mode, d0.ntiles);
  if (mode == PLAN_PRECOMP_DENSE) {
    CHECK(d0.gshape == GSHAPE_TILE, "dense grid on super tiles");
    CHECK(P.wg[f64 ? S_GRAM_F64 : d0.gop == GOP_F16PAIR ? S_GRAM_F32 : S_GRAM_BF16] == tiles,
          "dense Gram grid");
  }
  if (precomp) {
    // k_precomp reads Z columns below ceil((B + 1) / 64) * 64 and writes strip sums of the
    // columns up to B; k_precomp_stat writes B + 1 statistics
    const int64_t cols = (r.B + 1 + 63) / 64 * 64;
    CHECK(cols <= d0.B_pad, "precomp columns %lld > B_pad %lld", (long long)cols,
          (long long)d0.B_pad);
    need[B_Z] = (size_t)d0.nt * TILE_WORDS * d0.B_pad * 4;
    need[B_PART] = (size_t)d0.ntiles * PC_STRIPS * 3 * d0.B_pad * 8;
    need[B_PSTAT] = (size_t)(r.B + 1) * 8;
  }
  for (int k = 0; k < B_PERMOUT; ++k) {
    CHECK(P.size[k] >= need[k], "mode %d buffer %d: %zu < %zu", mode, k, P.size[k], need[k]);
    CHECK(P.off[k] + P.size[k] <= P.bytes, "mode %d buffer %d past the region", mode, k);
    for (int m = 0; m < k; ++m) {
      if (P.size[k] == 0 || P.size[m] == 0) continue;
      const bool apart = P.off[k] + P.size[k] <= P.off[m] || P.off[m] + P.size[m] <= P.off[k];
      CHECK(apart, "mode %d buffers %d and %d overlap", mode, k, m);
    }
  }
  CHECK(P.size[B_PLANES] == 0, "mode %d keeps centred planes", mode);
  for (int k : {S_CENTER_F64, S_CENTER_SPLIT, S_PERM_F64, S_PERM_S2, S_PERM_S3, S_PSTAT})
    CHECK(P.wg[k] == 0, "mode %d launches slot %d", mode, k);
  CHECK((P.wg[S_MEMBER] > 0) == precomp, "mode %d split stream", mode);
  CHECK(P.bytes < make_plan(r).bytes || r.B == 0 || precomp,
        "blocks-only plan not smaller than the full plan");
}

// Row units of the resampling stage: rowk_coords against a plain enumeration (row by row,
// kc tiles at a time); together the units cover every stored tile (i <= j) exactly once.
static void check_row_units() {
  for (int nt = 1; nt <= 80; ++nt)
    for (int kc = 1; kc <= 40; ++kc) {
      TestDesc d{};
      d.nt = nt;
      d.kc = kc;
      int u = 0;
      for (int i = 0; i < nt; ++i)
        for (int j0 = i; j0 < nt; j0 += kc, ++u) {
          int gi, g0, g1;
          rowk_coords(d, u, &gi, &g0, &g1);
          const int e = j0 + kc < nt ? j0 + kc : nt;
          CHECK(gi == i && g0 == j0 && g1 == e, "nt %d kc %d unit %d: (%d,%d,%d) vs (%d,%d,%d)",
                nt, kc, u, gi, g0, g1, i, j0, e);
        }
      int nrk = 0;
      for (int i = 0; i < nt; ++i) nrk += (nt - i + kc - 1) / kc;
      CHECK(u == nrk, "nt %d kc %d: %d units enumerated, %d counted", nt, kc, u, nrk);
    }
}

// Requests at and past the largest tile grid: the planner's tile counts and footprints are
// formed in 64 bits and never wrap; grids past MAX_TILE_GRID and launches past what one
// dispatch addresses are rejected as invalid (nothing here touches a device).
static void check_large_grids() {
  auto req = [](int64_t nx, int64_t ny, int64_t p, int64_t B, int prec) {
    etest_request r{};
    r.kind = ETEST_ED;
    r.prec = prec;
    r.nx = nx;
    r.ny = ny;
    r.p = p;
    r.B = B;
    r.seed = 1;
    r.X = (const void*)0x1000;
    r.Y = (const void*)0x2000;
    return r;
  };
  const int64_t T = TILE;
  // nt = 46340 (accepted), 46341, 65536 and n = 2^31 - 1 (rejected), at p = 1
  {
    const etest_request r = req(23170 * T, 23170 * T, 1, 100, ETEST_PREC_F32);
    CHECK(validate_request(r) == ETEST_OK, "nt = 46340 rejected");
    const TestPlan P = make_plan(r);
    const int64_t nt = 46340, ntiles = nt * (nt + 1) / 2;
    CHECK(P.d.nt == nt && P.d.ntiles == ntiles, "ntiles %lld != %lld", (long long)P.d.ntiles,
          (long long)ntiles);
    CHECK(P.size[B_D] == (size_t)ntiles * T * T * 4, "D bytes %zu", P.size[B_D]);
    CHECK(P.bytes > (size_t)ntiles * T * T * 8, "footprint %zu wrapped", P.bytes);
    int64_t fp = 0;
    CHECK(etest_footprint(&r, &fp) == ETEST_OK && fp > (int64_t)70e12, "footprint %lld",
          (long long)fp);
    // the last stored tile's index and the middle row's first tile, formed in 64 bits
    CHECK(tile_index((int)nt - 1, (int)nt - 1, (int)nt) == ntiles - 1, "last tile index");
    const int64_t i = nt / 2;
    CHECK(tile_index((int)i, (int)i, (int)nt) == i * nt - i * (i - 1) / 2, "middle tile index");
    // its Gram launch (one workgroup per stored tile) exceeds one dispatch's 2^32 work-items
    Batch b;
    CHECK(build_batch(&r, 1, false, &b) == ETEST_EINVAL, "nt = 46340 batch accepted");
  }
  // the largest grids whose launches fit: every slot's grid below 2^31 workgroups and 2^32
  // work-items (the Gram's 256-thread workgroups allow nt(nt+1)/2 < 2^24)
  for (const int64_t nt : {(int64_t)2000, (int64_t)5791}) {
    const etest_request r = req(nt / 2 * T, (nt - nt / 2) * T, 1, 1000, ETEST_PREC_F32);
    Batch b;
    CHECK(build_batch(&r, 1, false, &b) == ETEST_OK, "nt = %lld rejected: %s", (long long)nt,
          etest_last_error());
    if (!b.plans.empty()) {
      // one workgroup per stored tile, or per 2 x 2 super tile of the ceil(nt / 2) grid
      const int64_t st = (nt + 1) / 2;
      const TestPlan& P = b.plans[0];
      const bool tiles = P.wg[S_GRAM_F32] == nt * (nt + 1) / 2 && P.wg[S_GRAM_F32S] == 0;
      const bool supers = P.wg[S_GRAM_F32S] == st * (st + 1) / 2 && P.wg[S_GRAM_F32] == 0 &&
                          P.wg[S_GRAM_FIN] == nt * (nt + 1) / 2;
      CHECK(tiles || supers, "gram grid of nt = %lld", (long long)nt);
      const int64_t ntl = nt * (nt + 1) / 2;  // stored tiles: two workgroups each up to 2^22
      CHECK(P.wg[S_CENTER_SPLIT] == ntl * (ntl <= (1 << 22) ? 2 : 1), "centring grid of nt = %lld",
            (long long)nt);
    }
  }
  for (const int64_t n : {(int64_t)46341 * T, (int64_t)65536 * T, (int64_t)2147483647})
    for (int prec : {ETEST_PREC_F64, ETEST_PREC_F32, ETEST_PREC_BF16_REFINED}) {
      const etest_request r = req(n / 2, n - n / 2, 1, 10, prec);
      CHECK(validate_request(r) == ETEST_EINVAL, "n = %lld accepted", (long long)n);
      int64_t fp = -7;
      CHECK(etest_footprint(&r, &fp) == ETEST_EINVAL && fp == -7, "footprint of n = %lld",
            (long long)n);
      Batch b;
      CHECK(build_batch(&r, 1, false, &b) == ETEST_EINVAL, "batch of n = %lld", (long long)n);
    }
  // a valid grid whose resampling launch exceeds one dispatch (2^32 work-items): EINVAL
  {
    const etest_request r = req(20000, 20000, 10, 2000000000, ETEST_PREC_BF16_REFINED);
    CHECK(validate_request(r) == ETEST_OK, "large-B request rejected by validation");
    Batch b;
    CHECK(build_batch(&r, 1, false, &b) == ETEST_EINVAL, "oversized resampling launch accepted");
  }
  // tuned row units of one tile on a large FP64 grid: row-unit count past 2^31 is rejected
  {
    const etest_request r = req(20000 * T, 20000 * T, 1, 0, ETEST_PREC_F64);
    const TestPlan P = make_plan(r, 1);
    CHECK(P.d.n_rowk == 2147483647, "n_rowk not saturated: %d", P.d.n_rowk);
    CHECK(check_launch_sizes(&P, 1) == ETEST_EINVAL, "saturated row units accepted");
  }
}

// Split-stream width: 16 splits per workgroup for a launch the chip holds at once, 32 for a
// larger one, with every test's grid share counted in that width.
static void check_member_width() {
  auto req = [](int64_t nx, int64_t ny, int64_t B, const void* x) {
    etest_request r{};
    r.kind = ETEST_ED;
    r.prec = ETEST_PREC_F32;
    r.nx = nx;
    r.ny = ny;
    r.p = 100;
    r.B = B;
    r.seed = 3;
    r.X = x;
    r.Y = (const char*)x + 0x100000;
    return r;
  };
  {
    Batch b;
    const etest_request r = req(2000, 2000, 10000, (const void*)0x1000);
    CHECK(build_batch(&r, 1, false, &b) == ETEST_OK, "one test");
    CHECK(!b.member_wide && b.plans[0].wg[S_MEMBER] == b.plans[0].d.B_pad / MEMBER_SPLITS,
          "one test of B = 10^4: %lld split workgroups", (long long)b.plans[0].wg[S_MEMBER]);
  }
  {
    std::vector<etest_request> rs;
    for (int t = 0; t < 256; ++t) rs.push_back(req(50 + 5 * t, 1500 - 5 * t, 2000, (const void*)(uintptr_t)(0x1000000 * (t + 1))));
    Batch b;
    CHECK(build_batch(rs.data(), (int64_t)rs.size(), false, &b) == ETEST_OK, "256 tests");
    CHECK(b.member_wide, "256 tests of B = 2000: narrow split stream");
    for (const TestPlan& P : b.plans)
      CHECK(P.wg[S_MEMBER] == P.d.B_pad / MEMBER_SPLITS_WIDE, "wide share %lld of B_pad %lld",
            (long long)P.wg[S_MEMBER], (long long)P.d.B_pad);
  }
}

int main() {
  check_member_width();
  check_row_units();
  check_large_grids();
  const int precs[3] = {ETEST_PREC_F64, ETEST_PREC_F32, ETEST_PREC_BF16_REFINED};
  const int64_t shapes[][4] = {{1, 1, 1, 0},       {1, 5, 3, 40},       {100, 100, 10, 1000},
                               {129, 127, 64, 255}, {2000, 2000, 1000, 10000},
                               {5000, 4000, 4096, 10000}, {20000, 20000, 2000, 10000},
                               {7, 300, 2, 1},      {50, 1500, 500, 2000}};
  for (const auto& sh : shapes)
    for (int prec : precs)
      for (int kind = 0; kind < 2; ++kind)
        for (int internal = 0; internal < 2; ++internal)
          for (int with_out = 0; with_out < 2; ++with_out) {
            etest_request r{};
            r.kind = kind;
            r.prec = prec;
            r.nx = sh[0];
            r.ny = sh[1];
            r.p = sh[2];
            r.B = sh[3];
            r.seed = 1;
            r.gamma = 0.5;
            r.X = (const void*)0x1000;
            r.Y = (const void*)0x2000;
            r.perm_stats = with_out ? (double*)0x3000 : nullptr;
            check_plan(r, internal != 0);
            if (!internal && !with_out) {
              check_mode_plan(r, PLAN_BLOCKS);
              check_mode_plan(r, PLAN_PRECOMP);
              check_mode_plan(r, PLAN_PRECOMP_DENSE);
            }
          }
  // one-sample plans of the HSIC test (ny = 0: the Gram covers the rows of one sample)
  for (int64_t n : {4, 127, 128, 129, 1000, 4096})
    for (int prec : precs) {
      etest_request r{};
      r.kind = ETEST_MMD;
      r.prec = prec;
      r.nx = n;
      r.ny = 0;
      r.p = 37;
      r.gamma = 0.1;
      r.X = r.Y = (const void*)0x1000;
      check_mode_plan(r, PLAN_BLOCKS);
      const TestPlan P = make_plan(r, 0, PLAN_BLOCKS);
      CHECK(P.d.ty == 0 && P.d.nt == P.d.tx && P.d.tx * TILE >= n, "one-sample tiles n %lld",
            (long long)n);
    }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
