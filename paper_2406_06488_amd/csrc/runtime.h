// Host runtime shared by the synchronous, batched and serving entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <mutex>
#include <vector>

#include "common.h"
#include "etest.h"

namespace et {

// Kernel launchers (defined next to their kernels).
void launch_clear_flags(hipStream_t st, const TestDesc* d, const int64_t* offs, int n);
void launch_colpart(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n);
void launch_colmean(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n);
void launch_stage(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n);
void launch_cross_final(hipStream_t st, const TestDesc* d);
// super_tiles: the 256 x 256 kernel, which writes the raw Gram tiles only; the block values
// then come from launch_gram_finish (one workgroup per stored tile)
void launch_gram(int gop, bool super_tiles, int64_t blocks, hipStream_t st, const TestDesc* d,
                 const int64_t* offs, int n, bool dual = false);
void launch_gram_finish(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs,
                        int n, bool dual);
void launch_rowsum(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n);
void launch_observed(hipStream_t st, const TestDesc* d, const int64_t* sel, int n);
void launch_center(bool f64, int64_t blocks, hipStream_t st, const TestDesc* d,
                   const int64_t* offs, int n);
// A split-stream launch of more workgroups than MI355X holds at once (8 per CU of 256) at
// MEMBER_SPLITS per workgroup runs MEMBER_SPLITS_WIDE per workgroup instead.
constexpr int64_t MEMBER_WIDE_MIN_WG = 8 * 256;
// wide: MEMBER_SPLITS_WIDE split columns per workgroup (the launch table must count them so)
void launch_member(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n,
                   bool wide = false);
void launch_member_public(int64_t nx, int64_t ny, uint64_t seed, int64_t b0, int64_t count,
                          uint32_t* words, hipStream_t st);
void launch_member_import(int64_t bpad, hipStream_t st, const TestDesc* d, const uint32_t* w);
void launch_perm(int variant, int64_t blocks, hipStream_t st, const TestDesc* d,
                 const int64_t* offs, int ntests, const int32_t* pcr);
void launch_pstat(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n);
void launch_rowmap(const uint32_t* words, int64_t count, int64_t maps, int64_t n, int64_t nx,
                   int32_t* rowmap, hipStream_t st);
void launch_collect(const TestDesc* d, int m, int64_t c0, int64_t B, double* stats,
                    int32_t* flags, hipStream_t st);
void launch_count(const double* stats, int64_t B, const int32_t* flags, double* perm_out,
                  DevResult* result, hipStream_t st);
void launch_precomp(bool f64, const TestDesc* d, int64_t ntiles, int64_t B, double* part,
                    hipStream_t st);
void launch_precomp_stat(const TestDesc* d, int64_t ntiles, int64_t B, const double* part,
                         double* stats, hipStream_t st);
void launch_permgen(int64_t n, uint64_t seed, int64_t b0, int64_t count, int64_t total,
                    int32_t* perms, hipStream_t st);
void launch_hsic_prep(bool f64, const TestDesc* d, int64_t n, void* kx, void* ky, double* rx,
                      double* ry, double* hs, int32_t* flags, hipStream_t st);
void launch_hsic_terms(bool f64, const void* kx, const void* ky, int64_t n, const int32_t* perms,
                       int64_t nperm, const double* rx, const double* ry, double* part,
                       hipStream_t st);
void launch_hsic_stat(const double* part, int64_t n, int64_t nperm, const double* hs,
                      double* stats, hipStream_t st);
void launch_unpack(bool f64, int64_t elems, hipStream_t st, const TestDesc* d, void* xx, void* yy,
                   void* xy);

// Resampling workgroups of a test for pcn split-column chunks: one per (row range,
// group of up to cc chunks).
inline int64_t perm_units(const TestDesc& d, int pcn) {
  return (int64_t)d.n_rowk * ((pcn + d.cc - 1) / d.cc);
}

// Launch slots: one prefix array of workgroup counts per slot.
enum Slot {
  S_COLPART, S_COLMEAN, S_STAGE, S_GRAM_F64, S_GRAM_F32, S_GRAM_BF16, S_GRAM_F32S,
  S_GRAM_BF16S, S_GRAM_FIN, S_MEMBER, S_ROWSUM,
  S_CENTER_F64, S_CENTER_SPLIT, S_PERM_F64, S_PERM_S2, S_PERM_S3, S_PSTAT, S_COUNT
};

// Every Gram slot of a launch table: FP64 rows, fp16 pairs and BF16 operands, in 128-tile
// and super-tile workgroups, then the finish of the super-tile Gram (one workgroup per
// stored tile).  offs(slot): device launch table; total(slot): its workgroups.
template <class Offs, class Total>
inline void launch_gram_slots(Offs offs, Total total, hipStream_t st, const TestDesc* D, int n,
                              bool dual) {
  launch_gram(GOP_F64, false, total(S_GRAM_F64), st, D, offs(S_GRAM_F64), n, dual);
  launch_gram(GOP_F16PAIR, false, total(S_GRAM_F32), st, D, offs(S_GRAM_F32), n, dual);
  launch_gram(GOP_BF16, false, total(S_GRAM_BF16), st, D, offs(S_GRAM_BF16), n, dual);
  launch_gram(GOP_F16PAIR, true, total(S_GRAM_F32S), st, D, offs(S_GRAM_F32S), n, dual);
  launch_gram(GOP_BF16, true, total(S_GRAM_BF16S), st, D, offs(S_GRAM_BF16S), n, dual);
  launch_gram_finish(total(S_GRAM_FIN), st, D, offs(S_GRAM_FIN), n, dual);
}
constexpr int GRAM_SLOTS[] = {S_GRAM_F64, S_GRAM_F32, S_GRAM_BF16, S_GRAM_F32S, S_GRAM_BF16S,
                              S_GRAM_FIN};

// Buffer ids inside one test's region.
enum Buf { B_COLPART, B_COLMEAN, B_W, B_NRM, B_D, B_TSUM, B_TMAX, B_RSUM, B_OBS, B_PLANES, B_Z,
           B_PART, B_PSTAT, B_FLAGS, B_RESULT, B_PERMOUT, B_NBUF };

struct TestPlan {
  TestDesc d{};              // sizes now, pointers once the workspace is placed
  size_t bytes = 0;          // workspace bytes of this test
  size_t off[B_NBUF] = {};   // offsets of its buffers inside its region
  size_t size[B_NBUF] = {};  // their sizes in bytes
  bool internal_perm = false;  // per-split output lives in the region (off[B_PERMOUT])
  int partner = -1;          // ED test: index of the MMD test whose blocks its Gram writes
  bool share_z = false;      // ... and whose split stream it provides
  int64_t wg[S_COUNT] = {};  // workgroups per launch slot
};

// Sets the calling thread's error message; returns the status.
etest_status set_error(etest_status s, const std::string& msg);
etest_status validate_request(const etest_request& r);
// EINVAL when a launch of the plans would exceed what one dispatch can address.
etest_status check_launch_sizes(const TestPlan* plans, size_t n);
// Plan modes: the efficient test; blocks and observed statistic only (one recomputation of
// the standard test); pooled blocks, split stream and the pre-computation test's buffers.
// PLAN_PRECOMP: the pre-computation test on the symmetric upper tiles; PLAN_PRECOMP_DENSE:
// the same test on the dense pooled matrix (every tile of the nt x nt grid).
enum PlanMode { PLAN_EFFICIENT = 0, PLAN_BLOCKS = 1, PLAN_PRECOMP = 2, PLAN_PRECOMP_DENSE = 3 };
TestPlan make_plan(const etest_request& r, int64_t kc_override = 0, int mode = PLAN_EFFICIENT);

// A set of tests laid out in one device workspace, ready to launch.
struct Batch {
  std::vector<TestPlan> plans;
  std::vector<TestDesc> descs;   // with device pointers
  std::vector<int64_t> offs;     // [S_COUNT][n + 1]
  void* ws = nullptr;            // device workspace
  size_t ws_bytes = 0;
  TestDesc* d_descs = nullptr;
  int64_t* d_offs = nullptr;
  DevResult* d_results = nullptr;
  double* d_perm = nullptr;      // internal perm-stat buffers (host-output calls)
  std::vector<size_t> base;      // each test's region offset inside ws
  // ws comes from the stream's cached workspace (stream_workspace) and is not freed with
  // the batch
  bool cached = false;
  // held while a cached workspace's pass is enqueued, so that concurrent callers on one
  // stream cannot interleave their launches over the same workspace (released by
  // free_batch)
  std::unique_lock<std::mutex> ws_hold;
  // single test: the descriptor and launch table go to the device as kernel arguments
  // (launch_put_desc, which also clears the flag words) instead of two host copies
  bool desc_by_kernel = false;
  // several tests: descriptors and launch tables go up in one copy from a pinned staging
  // slot (pinned_slot) instead of two copies from pageable host memory
  bool desc_pinned = false;
  // split stream of MEMBER_SPLITS_WIDE columns per workgroup (build_batch decides)
  bool member_wide = false;
};

// Device address and size of this GPU's no-allocation scratch array (k_noalloc.hip).
etest_status scratch_region(void** ptr, size_t* bytes);
void launch_put_desc(const TestDesc& d, const int64_t* offs, TestDesc* dd, int64_t* doffs,
                     hipStream_t st);
// Point a plan's descriptor at its buffers inside a device region.
void assign_pointers(TestPlan& P, char* region, DevResult* result);
// ED / MMD pairs of a request list that share staging and Gram: partner[s] = t when the
// ED test s feeds the MMD test t (same X, Y pointers, shapes and precision), else -1.
// share_z[s]: the pair also has the same seed and B, so t reads s's split stream.
struct Pairing {
  std::vector<int> partner;
  std::vector<char> share_z;
};
Pairing pair_tests(const etest_request* reqs, int64_t n);
// Fill the ED tests' pointers to their partners' buffers (descriptors already placed).
void link_partners(TestDesc* descs, const Pairing& pairing);
void init_pool_once();

// Build plans + layout (host only).  extra_perm: allocate internal perm-stat
// outputs for tests whose request has perm_stats == NULL but the caller wants them.
etest_status build_batch(const etest_request* reqs, int64_t n, bool internal_perm, Batch* b);
// Allocate the workspace on `st`, copy descriptors.
etest_status place_batch(Batch* b, hipStream_t st, bool stream_ordered);
// Optional stage events: begin[k] / end[k] bracket stage k on the stream it runs on.
constexpr int NSTAGE = 7;
struct StageEvents {
  hipEvent_t begin[NSTAGE], end[NSTAGE];
  uint32_t mask = 0;  // stages (bit k = stage k) whose events are recorded
};

// Optional second stream for the split stream, which does not depend on the data:
// it is forked after the descriptor copy and joined before the resampling stage.
struct Fork {
  hipStream_t aux;
  hipEvent_t start, done;
};

// Enqueue every stage of n tests whose descriptors (D) and launch tables (d_offs, with the
// same tables on the host in h_offs: [S_COUNT][n + 1] prefix sums of workgroups) are in
// device memory.  dual: some ED test also writes its MMD partner's blocks.  import_words:
// caller splits for a single test of B_pad import_bpad (or null).
// clear_flags false: the flag words were cleared already (launch_put_desc).
void enqueue_stages(const TestDesc* D, const int64_t* d_offs, const int64_t* h_offs, int n,
                    bool dual, hipStream_t st, const uint32_t* import_words, int64_t import_bpad,
                    const StageEvents* ev, const Fork* fork, bool clear_flags = true,
                    bool member_wide = false);
// Enqueue every stage.  import_words: caller splits for a single test (or null).
void enqueue_batch(const Batch& b, hipStream_t st, const uint32_t* import_words = nullptr,
                   const StageEvents* events = nullptr, const Fork* fork = nullptr);
void free_batch(Batch* b, hipStream_t st, bool stream_ordered);
etest_status dev_to_result(const DevResult& r, etest_result* out);

}  // namespace et
