// Fixed device scratch of the no-allocation entry point (etest_run_async_noalloc).
//
// The whole workspace of one test -- its descriptor, launch tables, result slot and every
// buffer its kernels index (staged rows, norms, blocks, tile sums, planes, split words,
// partial sums, statistics, flags) -- is placed in one file-scope device array instead of
// a stream-ordered allocation.  Each GPU the library runs on holds its own copy of the
// array until the process ends; its device address is taken once per device with
// hipGetSymbolAddress (the array's name in host code is only a host-side stand-in).
// Calls on one GPU share the array and race if they overlap; every kernel of the path
// writes what it later reads (flags are cleared by a kernel), so stale contents from a
// previous call are never read.
#include <mutex>

#include "runtime.h"

namespace et {

constexpr size_t SCRATCH_BYTES = (size_t)128 << 20;  // 128 MiB per GPU
constexpr int SCRATCH_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// One test's descriptor and launch tables, passed by value as kernel arguments so that
// no host buffer has to outlive the call and no copy node is enqueued.
struct DescArgs {
  TestDesc d;
  int64_t offs[S_COUNT * 2];
};

// It also clears the test's flag words, which every later kernel of the pass may update.
__global__ void k_put_desc(DescArgs a, TestDesc* __restrict__ dd, int64_t* __restrict__ doffs) {
  const int t = threadIdx.x;
  if (t == 0) *dd = a.d;
  if (t < S_COUNT * 2) doffs[t] = a.offs[t];
  if (t < FLAG_WORDS) a.d.flags[t] = 0;
}

etest_status scratch_region(void** ptr, size_t* bytes) {
  static std::mutex mu;
  static void* addr[SCRATCH_MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string("no device: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return set_error(ETEST_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(ETEST_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = SCRATCH_BYTES;
  return ETEST_OK;
}

void launch_put_desc(const TestDesc& d, const int64_t* offs, TestDesc* dd, int64_t* doffs,
                     hipStream_t st) {
  DescArgs a;
  a.d = d;
  for (int k = 0; k < S_COUNT * 2; ++k) a.offs[k] = offs[k];
  hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, st, a, dd, doffs);
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace et

using namespace et;

// One test on device buffers, enqueued on `stream` with the workspace in the scratch array:
// no device, pinned or stream-ordered allocation, no stream or event creation.  The same
// kernels, in the same order, as ed_test_async / mmd_test_async, on the caller's stream
// alone (the split stream is not forked).
extern "C" etest_status etest_run_async_noalloc(const etest_request* req, etest_result* d_out,
                                                void* stream) {
  if (!req || !d_out) return set_error(ETEST_EINVAL, "NULL argument");
  etest_status s = validate_request(*req);
  if (s != ETEST_OK) return s;
  TestPlan P = make_plan(*req);
  s = check_launch_sizes(&P, 1);
  if (s != ETEST_OK) return s;
  void* base = nullptr;
  size_t cap = 0;
  s = scratch_region(&base, &cap);
  if (s != ETEST_OK) return s;
  const size_t desc_bytes = align256(sizeof(TestDesc));
  const size_t offs_bytes = align256(sizeof(int64_t) * S_COUNT * 2);
  const size_t res_bytes = align256(sizeof(DevResult));
  const size_t total = desc_bytes + offs_bytes + res_bytes + P.bytes;
  if (total > cap)
    return set_error(ETEST_ENOMEM, "test needs " + std::to_string(total) +
                                       " bytes of workspace; the no-allocation scratch holds " +
                                       std::to_string(cap));
  char* w = (char*)base;
  TestDesc* dd = (TestDesc*)w;
  int64_t* doffs = (int64_t*)(w + desc_bytes);
  DevResult* dres = (DevResult*)(w + desc_bytes + offs_bytes);
  assign_pointers(P, w + desc_bytes + offs_bytes + res_bytes, dres);
  int64_t ho[S_COUNT * 2];
  for (int k = 0; k < S_COUNT; ++k) {
    ho[2 * k] = 0;
    ho[2 * k + 1] = P.wg[k];
  }
  hipStream_t st = (hipStream_t)stream;
  P.d.out6 = (double*)d_out;  // the final kernel writes the result there too
  launch_put_desc(P.d, ho, dd, doffs, st);
  enqueue_stages(dd, doffs, ho, 1, false, st, nullptr, 0, nullptr, nullptr, false);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ETEST_EDEVICE, std::string("enqueue: ") + hipGetErrorString(e));
  return ETEST_OK;
}
