// Standalone reduction that allocates nothing, for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// Its kernels are those of upir_reduce; the reduction scratch they need (a
// 256-byte header with the dynamic-schedule counters, then one 128-byte
// combine slot per workgroup) lives in one file-scope device array per GPU,
// sized for UPIR_REDUCE_NOALLOC_MAX_TEAMS workgroups. Host code never passes
// the array's name to a kernel or a copy: the array's device address is
// looked up once per device when a context opens (the device current) and
// kept; the kernels get that address.
//
// Every call on one GPU shares its array and leaves it as the call's kernels
// left it; each call first clears the header and the slots it will use with
// a small fill kernel (not a memset node, so a captured graph replays it
// correctly). Calls that can run at the same time on one GPU (other streams,
// other contexts, other host threads) race on the array.
#include <algorithm>
#include <mutex>

#include "runtime_internal.h"

namespace {

constexpr int64_t kMaxTeams = UPIR_REDUCE_NOALLOC_MAX_TEAMS;
constexpr size_t kScratchBytes = SCR_SLOTS + (size_t)kMaxTeams * 8 * upir::SLOT_WORDS;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

// Zero the header words, set the slot words to the empty pattern.
__global__ void k_clear_scratch(unsigned long long *p, int64_t header_words, int64_t total_words,
                                unsigned long long slot_value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total_words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = i < header_words ? 0ULL : slot_value;
}

}  // namespace

namespace upir {

hipError_t noalloc_setup(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace upir

extern "C" upir_status upir_reduce_noalloc(upir_ctx *c, int32_t op, int32_t dtype, const void *dev_in, int64_t n,
                                           const upir_spmd *spmd, const upir_sched *sched, upir_reduction *red) {
  using namespace upir;
  if (!c) return UPIR_EINVAL;
  if (!red || !red->result) return upir_fail(c, UPIR_EINVAL, "reduce_noalloc: result");
  if (red->result_on_host)
    return upir_fail(c, UPIR_EINVAL, "reduce_noalloc: the result must be a device address");
  if (op < UPIR_RED_SUM || op > UPIR_RED_MIN) return upir_fail(c, UPIR_EINVAL, "reduce_noalloc: op");
  if (dtype < UPIR_DT_F32 || dtype > UPIR_DT_I64) return upir_fail(c, UPIR_EINVAL, "reduce_noalloc: dtype");
  if (n < 0 || (n > 0 && !dev_in)) return upir_fail(c, UPIR_EINVAL, "reduce_noalloc: input");
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
  if (!c->noalloc_scratch) return upir_fail(c, UPIR_ESTATE, "reduce_noalloc: no scratch on this device");
  upir_loop L{};
  L.collapse = 1;
  L.dim[0] = upir_dim{0, n, 1};
  upir_sum_args a{dev_in, dtype, 0};
  upir_body b{UPIR_BODY_SUM, 1, &a, sizeof a};
  upir_reduction r = *red;
  r.op = op;
  r.async = 0;
  upir_sched s{};
  s.policy = UPIR_SCHED_AUTO;
  if (sched) s = *sched;
  upir_loop_obj lo;  // a loop description on the stack; its scratch is the static array
  upir_status st = describe_loop(c, &L, &s, &b, &r, &lo);
  if (st) return st;
  lo.scratch = (unsigned char *)c->noalloc_scratch;
  lo.part_cap = kMaxTeams;
  Plan pl;
  c->no_alloc = true;  // AUTO: tuned table or default, not the cost model
  st = resolve_plan(c, spmd, &lo, pl);
  c->no_alloc = false;
  if (st) return st;
  if (pl.S.T > kMaxTeams)
    return upir_fail(c, UPIR_EINVAL, "reduce_noalloc: %d workgroups exceed the maximum of %lld", pl.S.T,
                     (long long)kMaxTeams);
  const int64_t header_words = SCR_SLOTS / 8;
  const int64_t total_words = header_words + (int64_t)pl.S.T * SLOT_WORDS;
  const unsigned long long empty = red_is_int(&lo) ? 0ULL : ~0ULL;
  const int blocks = (int)std::min<int64_t>((total_words + 255) / 256, 256);
  hipLaunchKernelGGL(k_clear_scratch, dim3(blocks), dim3(256), 0, c->stream, (unsigned long long *)lo.scratch,
                     header_words, total_words, empty);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return upir_hipfail(c, e, "reduce_noalloc: scratch clear");
  return launch_plan(c, &lo, pl, false);
}
