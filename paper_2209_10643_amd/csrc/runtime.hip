// libupir host runtime: contexts, the data table (sec. 4), loop handles and
// SPMD launches (sec. 3.1, 3.2), reductions (sec. 5) and graph replay.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "runtime_internal.h"

using namespace upir;

// ------------------------------------------------------------------ errors
upir_status upir_fail(upir_ctx *c, upir_status s, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

upir_status upir_hipfail(upir_ctx *c, hipError_t e, const char *what) {
  return upir_fail(c, UPIR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPTRY(c, expr)                                   \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return upir_hipfail(c, e_, #expr); \
  } while (0)

extern "C" const char *upir_strerror(upir_status s) {
  switch (s) {
    case UPIR_OK: return "ok";
    case UPIR_EINVAL: return "invalid argument";
    case UPIR_ENOTMAPPED: return "host pointer not mapped";
    case UPIR_EOVERLAP: return "mapping overlaps an existing mapping";
    case UPIR_ENOMEM: return "out of memory";
    case UPIR_EHIP: return "HIP runtime error";
    case UPIR_EUNSUPPORTED: return "unsupported";
    case UPIR_EDEPEND: return "task dependence error";
    case UPIR_ESTATE: return "invalid state";
  }
  return "unknown status";
}

extern "C" const char *upir_last_error(const upir_ctx *c) { return c ? c->err.c_str() : "no context"; }

extern "C" const char *upir_version(void) { return "upir-mi355x 0.1 (gfx950)"; }

// --------------------------------------------------------------- allocator
void *upir_dalloc(upir_ctx *c, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (c->alloc) return c->alloc(bytes, c->user);
  if (c->none) return nullptr;
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void upir_dfree(upir_ctx *c, void *p) {
  if (!p) return;
  if (c->free_fn) {
    c->free_fn(p, c->user);
    return;
  }
  if (!c->none) (void)hipFree(p);
}

extern "C" upir_status upir_set_allocator(upir_ctx *c, upir_alloc_fn a, upir_free_fn f, void *user) {
  if (!c) return UPIR_EINVAL;
  if ((a == nullptr) != (f == nullptr)) return upir_fail(c, UPIR_EINVAL, "allocator and deallocator go together");
  if (!c->table.empty() || !c->loops.empty())
    return upir_fail(c, UPIR_ESTATE, "allocator can only change while nothing is allocated");
  c->alloc = a;
  c->free_fn = f;
  c->user = user;
  return UPIR_OK;
}

// ----------------------------------------------------------------- context
extern "C" upir_status upir_init(int device, void *hip_stream, upir_ctx **out) {
  if (!out) return UPIR_EINVAL;
  *out = nullptr;
  upir_ctx *c = new (std::nothrow) upir_ctx();
  if (!c) return UPIR_ENOMEM;
  c->device = device;
  if (device == UPIR_DEVICE_NONE) {
    c->none = true;
    *out = c;
    return UPIR_OK;
  }
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    delete c;
    return UPIR_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return UPIR_EHIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->num_cus = prop.multiProcessorCount;
    c->max_lds = (int)prop.maxSharedMemoryPerMultiProcessor;
  }
  if (upir::noalloc_setup(device, &c->noalloc_scratch) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return UPIR_EHIP;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return UPIR_EHIP;
    }
    c->own_stream = true;
  }
  *out = c;
  return UPIR_OK;
}

static void free_loop(upir_ctx *c, upir_loop_obj *lp) {
  upir_dfree(c, lp->scratch);
  upir_dfree(c, lp->ws);
  delete lp;
}

extern "C" upir_status upir_finalize(upir_ctx *c) {
  if (!c) return UPIR_EINVAL;
  if (!c->none && c->stream) {
    if (!c->capturing) (void)upir::settle(c);
    (void)hipStreamSynchronize(c->stream);
  }
  for (auto *g : c->graphs) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (void *p : g->owned) upir_dfree(c, p);
    delete g;
  }
  for (auto *lp : c->loops) free_loop(c, lp);
  for (auto &kv : c->table) upir_dfree(c, kv.second.dev);
  upir_dfree(c, c->trace_clock);
  upir_dfree(c, c->fold_buf[0]);
  upir_dfree(c, c->fold_buf[1]);
  for (void *p : c->retired) upir_dfree(c, p);
  upir_model_free(c);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  for (hipStream_t cs : c->copy_stream)
    if (cs) (void)hipStreamDestroy(cs);
  delete c;
  return UPIR_OK;
}

extern "C" upir_status upir_sync(upir_ctx *c) {
  if (!c) return UPIR_EINVAL;
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "cannot synchronise during graph capture");
  upir_status st = upir::settle(c);
  if (st) return st;
  HIPTRY(c, hipStreamSynchronize(c->stream));
  return UPIR_OK;
}

// ------------------------------------------------------------- data table
static Mapping *find_containing(upir_ctx *c, uintptr_t h) {
  auto it = c->table.upper_bound(h);
  if (it == c->table.begin()) return nullptr;
  --it;
  Mapping &m = it->second;
  return (h >= m.host && h < m.host + m.bytes) ? &m : nullptr;
}

extern "C" upir_status upir_data_map(upir_ctx *c, void *host, size_t bytes, int32_t map, int32_t access,
                                     void **dev_out) {
  if (!c) return UPIR_EINVAL;
  if (!host || bytes == 0) return upir_fail(c, UPIR_EINVAL, "data_map: null host pointer or zero size");
  if (map < UPIR_MAP_TO || map > UPIR_MAP_ALLOC) return upir_fail(c, UPIR_EINVAL, "data_map: bad map type %d", map);
  if (access < UPIR_ACCESS_RO || access > UPIR_ACCESS_RW)
    return upir_fail(c, UPIR_EINVAL, "data_map: bad access %d", access);
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "data_map during graph capture");
  const uintptr_t h = (uintptr_t)host;
  if (h + bytes < h) return upir_fail(c, UPIR_EINVAL, "data_map: range wraps");
  if (Mapping *m = find_containing(c, h)) {
    if (h + bytes <= m->host + m->bytes) {
      m->refs++;
      if (dev_out) *dev_out = (char *)m->dev + (h - m->host);
      return UPIR_OK;
    }
    return upir_fail(c, UPIR_EOVERLAP, "data_map: [%p,+%zu) overlaps a mapping", host, bytes);
  }
  auto nx = c->table.upper_bound(h);
  if (nx != c->table.end() && nx->second.host < h + bytes)
    return upir_fail(c, UPIR_EOVERLAP, "data_map: [%p,+%zu) overlaps a mapping", host, bytes);
  if (c->none && map != UPIR_MAP_ALLOC)
    return upir_fail(c, UPIR_ESTATE, "data_map: copies need a device (host-only context)");
  void *dev = upir_dalloc(c, bytes);
  if (!dev) return upir_fail(c, UPIR_ENOMEM, "data_map: allocator returned NULL for %zu bytes", bytes);
  if (map == UPIR_MAP_TO || map == UPIR_MAP_TOFROM) {
    hipError_t e = hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
      upir_dfree(c, dev);
      return upir_hipfail(c, e, "data_map: host to device copy");
    }
  }
  c->table[h] = Mapping{h, bytes, dev, 1, map, access};
  if (dev_out) *dev_out = dev;
  return UPIR_OK;
}

extern "C" upir_status upir_data_unmap(upir_ctx *c, void *host, int32_t map) {
  if (!c) return UPIR_EINVAL;
  if (map < UPIR_MAP_TO || map > UPIR_MAP_ALLOC) return upir_fail(c, UPIR_EINVAL, "data_unmap: bad map type %d", map);
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "data_unmap during graph capture");
  auto it = c->table.find((uintptr_t)host);
  if (it == c->table.end()) return upir_fail(c, UPIR_ENOTMAPPED, "data_unmap: %p does not start a mapping", host);
  Mapping &m = it->second;
  if (m.refs == 1 && !c->none) {  // a deferred result may live in this buffer
    upir_status st = upir::settle(c);
    if (st) return st;
  }
  if (--m.refs > 0) return UPIR_OK;
  if (!c->none && (map == UPIR_MAP_FROM || map == UPIR_MAP_TOFROM) && m.access != UPIR_ACCESS_RO) {
    hipError_t e = hipMemcpyAsync(host, m.dev, m.bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      m.refs++;
      return upir_hipfail(c, e, "data_unmap: device to host copy");
    }
  } else if (!c->none) {
    // the buffer may still be read by queued work
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      m.refs++;
      return upir_hipfail(c, e, "data_unmap: synchronise");
    }
  }
  upir_dfree(c, m.dev);
  c->table.erase(it);
  return UPIR_OK;
}

upir_status upir_map_range(upir_ctx *c, const void *host, size_t *bytes, void **dev) {
  const uintptr_t h = (uintptr_t)host;
  Mapping *m = find_containing(c, h);
  if (!m) return upir_fail(c, UPIR_ENOTMAPPED, "%p not mapped", host);
  const size_t off = h - m->host;
  if (*bytes == 0) *bytes = m->bytes - off;
  if (off + *bytes > m->bytes) return upir_fail(c, UPIR_EINVAL, "range leaves its mapping");
  *dev = (char *)m->dev + off;
  return UPIR_OK;
}

extern "C" upir_status upir_data_update(upir_ctx *c, void *host, size_t bytes, int32_t dir) {
  if (!c) return UPIR_EINVAL;
  if (dir != UPIR_TO_DEVICE && dir != UPIR_FROM_DEVICE) return upir_fail(c, UPIR_EINVAL, "data_update: bad direction");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "data_update during graph capture");
  if (c->none) return upir_fail(c, UPIR_ESTATE, "data_update needs a device");
  const uintptr_t h = (uintptr_t)host;
  Mapping *m = find_containing(c, h);
  if (!m) return upir_fail(c, UPIR_ENOTMAPPED, "data_update: %p not mapped", host);
  const size_t off = h - m->host;
  if (bytes == 0) bytes = m->bytes - off;
  if (off + bytes > m->bytes) return upir_fail(c, UPIR_EINVAL, "data_update: range leaves its mapping");
  char *dev = (char *)m->dev + off;
  if (dir == UPIR_TO_DEVICE) {
    HIPTRY(c, hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c->stream));
  } else {
    upir_status st = upir::settle(c);
    if (st) return st;
    HIPTRY(c, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
  }
  return UPIR_OK;
}

extern "C" upir_status upir_data_lookup(upir_ctx *c, const void *host, void **dev_out) {
  if (!c || !dev_out) return UPIR_EINVAL;
  Mapping *m = find_containing(c, (uintptr_t)host);
  if (!m) return upir_fail(c, UPIR_ENOTMAPPED, "data_lookup: %p not mapped", host);
  *dev_out = (char *)m->dev + ((uintptr_t)host - m->host);
  return UPIR_OK;
}

static upir_status xlate(upir_ctx *c, upir_loop_obj *lp, const void *p, const void **out) {
  if (lp->args_dev || !p) {
    *out = p;
    return UPIR_OK;
  }
  Mapping *m = find_containing(c, (uintptr_t)p);
  if (!m) return upir_fail(c, UPIR_ENOTMAPPED, "loop body argument %p is not mapped", p);
  *out = (const char *)m->dev + ((uintptr_t)p - m->host);
  return UPIR_OK;
}

// ------------------------------------------------------------- loop handles
static int64_t trip(int64_t lb, int64_t ub, int64_t st) {
  if (st > 0) return ub > lb ? (ub - lb + st - 1) / st : 0;
  return lb > ub ? (lb - ub + (-st) - 1) / (-st) : 0;
}

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

static size_t args_size_of(int32_t kind) {
  switch (kind) {
    case UPIR_BODY_AXPY: return sizeof(upir_axpy_args);
    case UPIR_BODY_SUM: return sizeof(upir_sum_args);
    case UPIR_BODY_JACOBI5: return sizeof(upir_jacobi5_args);
    case UPIR_BODY_MATMUL_F32:
    case UPIR_BODY_MATMUL_BF16:
    case UPIR_BODY_MATMUL_SPLIT3: return sizeof(upir_matmul_args);
    case UPIR_BODY_MATVEC: return sizeof(upir_matvec_args);
    case UPIR_BODY_OWNER: return sizeof(upir_owner_args);
    case UPIR_BODY_COVER: return sizeof(upir_cover_args);
    case UPIR_BODY_FILTER7: return sizeof(upir_filter7_args);
  }
  return 0;
}

static bool is_matmul(int32_t k) {
  return k == UPIR_BODY_MATMUL_F32 || k == UPIR_BODY_MATMUL_BF16 || k == UPIR_BODY_MATMUL_SPLIT3;
}

extern "C" size_t upir_matmul_workspace_bytes(int32_t kind, int64_t M, int64_t N, int64_t K) {
  if (M < 0 || N < 0 || K < 0) return 0;
  // k is padded to the 32-wide panels one of the layouts uses
  if (kind == UPIR_BODY_MATMUL_BF16) return (size_t)(M + N) * upir::mm_kpad(K) * 2;
  if (kind == UPIR_BODY_MATMUL_SPLIT3) return (size_t)(M + N) * upir::mm_kpad(K) * 4;
  return 0;
}

static upir_status validate_sched(upir_ctx *c, const upir_loop &L, const upir_sched &S, int32_t kind) {
  if (S.policy < UPIR_SCHED_STATIC || S.policy > UPIR_SCHED_AUTO)
    return upir_fail(c, UPIR_EINVAL, "schedule policy %d", S.policy);
  if (S.distribute < UPIR_DIST_TEAMS_UNITS || S.distribute > UPIR_DIST_UNITS)
    return upir_fail(c, UPIR_EINVAL, "distribute %d", S.distribute);
  if ((S.policy == UPIR_SCHED_STATIC_CHUNK || S.policy == UPIR_SCHED_DYNAMIC || S.policy == UPIR_SCHED_GUIDED) &&
      S.chunk < 1)
    return upir_fail(c, UPIR_EINVAL, "chunk must be >= 1 for this policy");
  bool tiled = false;
  for (int d = 0; d < 3; ++d) {
    if (S.tile[d] < 0) return upir_fail(c, UPIR_EINVAL, "negative tile");
    if (S.tile[d] > 0) tiled = true;
  }
  if (tiled && S.policy != UPIR_SCHED_AUTO) {
    for (int d = 0; d < L.collapse; ++d) {
      if (S.tile[d] <= 0) return upir_fail(c, UPIR_EINVAL, "tile needs an extent for every collapsed dimension");
      if (L.dim[d].step != 1) return upir_fail(c, UPIR_EUNSUPPORTED, "tiled schedules need unit steps");
    }
    for (int d = L.collapse; d < 3; ++d)
      if (S.tile[d] != 0) return upir_fail(c, UPIR_EINVAL, "tile given for a dimension the loop does not have");
    if (S.tile[L.collapse - 1] % 4 != 0)
      return upir_fail(c, UPIR_EINVAL, "innermost tile extent must be a multiple of 4");
    if (S.policy == UPIR_SCHED_DYNAMIC || S.policy == UPIR_SCHED_GUIDED)
      return upir_fail(c, UPIR_EUNSUPPORTED, "dynamic / guided schedules are not tiled");
    if (S.distribute != UPIR_DIST_TEAMS_UNITS)
      return upir_fail(c, UPIR_EUNSUPPORTED, "tiled schedules distribute over teams and units");
    if (kind == UPIR_BODY_MATVEC) return upir_fail(c, UPIR_EUNSUPPORTED, "MATVEC rows are not tiled");
  }
  if (kind == UPIR_BODY_MATVEC && (S.policy == UPIR_SCHED_DYNAMIC || S.policy == UPIR_SCHED_GUIDED))
    return upir_fail(c, UPIR_EUNSUPPORTED, "MATVEC takes static schedules");
  return UPIR_OK;
}

// Validate a loop description and fill *lp from it: no allocation, nothing
// enqueued (scratch and workspace are the caller's business).
upir_status describe_loop(upir_ctx *c, const upir_loop *loop, const upir_sched *sched, const upir_body *body,
                          const upir_reduction *red, upir_loop_obj *lp) {
  if (!loop || !body) return upir_fail(c, UPIR_EINVAL, "loop_parallel: null loop or body");
  const upir_loop &L = *loop;
  if (L.collapse < 1 || L.collapse > 3) return upir_fail(c, UPIR_EINVAL, "collapse %d not in 1..3", L.collapse);
  int64_t cnt[3] = {1, 1, 1};
  __int128 n = 1;
  for (int d = 0; d < L.collapse; ++d) {
    if (L.dim[d].step == 0) return upir_fail(c, UPIR_EINVAL, "dimension %d has step 0", d);
    cnt[d] = trip(L.dim[d].lb, L.dim[d].ub, L.dim[d].step);
    n *= cnt[d];
  }
  if (n > ((__int128)1 << 62)) return upir_fail(c, UPIR_EINVAL, "trip count too large");
  const int32_t kind = body->kind;
  const size_t asz = args_size_of(kind);
  if (!asz) return upir_fail(c, UPIR_EINVAL, "unknown body kind %d", kind);
  if (!body->args || body->args_size != asz)
    return upir_fail(c, UPIR_EINVAL, "body args size %zu, expected %zu", body->args_size, asz);
  if ((kind == UPIR_BODY_AXPY || kind == UPIR_BODY_SUM || kind == UPIR_BODY_MATVEC) && L.collapse != 1)
    return upir_fail(c, UPIR_EINVAL, "this body runs a 1-D loop");
  if ((kind == UPIR_BODY_JACOBI5 || kind == UPIR_BODY_FILTER7 || is_matmul(kind)) && L.collapse != 2)
    return upir_fail(c, UPIR_EINVAL, "this body runs a collapse(2) loop");
  upir_sched S{};
  S.policy = UPIR_SCHED_AUTO;
  if (sched) S = *sched;
  upir_status st = validate_sched(c, L, S, kind);
  if (st) return st;
  upir_reduction R{};
  bool has_red = red && red->op != UPIR_RED_NONE;
  if (red) R = *red;
  if (red && (red->op < UPIR_RED_NONE || red->op > UPIR_RED_MIN)) return upir_fail(c, UPIR_EINVAL, "reduction op");
  if (kind == UPIR_BODY_SUM && !has_red) return upir_fail(c, UPIR_EINVAL, "SUM body needs a reduction");
  if (has_red && (is_matmul(kind) || kind == UPIR_BODY_OWNER || kind == UPIR_BODY_COVER || kind == UPIR_BODY_FILTER7))
    return upir_fail(c, UPIR_EINVAL, "this body has no value to reduce");
  if (has_red && !R.result) return upir_fail(c, UPIR_EINVAL, "reduction without a result address");
  int32_t sum_dtype = UPIR_DT_F32;
  if (kind == UPIR_BODY_SUM) {
    sum_dtype = ((const upir_sum_args *)body->args)->dtype;
    if (sum_dtype < UPIR_DT_F32 || sum_dtype > UPIR_DT_I64) return upir_fail(c, UPIR_EINVAL, "sum dtype");
  }
  int64_t M = 0, N = 0, K = 0;
  if (is_matmul(kind)) {
    const upir_matmul_args &a = *(const upir_matmul_args *)body->args;
    for (int d = 0; d < 2; ++d)
      if (L.dim[d].lb != 0 || L.dim[d].step != 1)
        return upir_fail(c, UPIR_EUNSUPPORTED, "matmul loops cover C from (0,0) with unit steps");
    M = cnt[0];
    N = cnt[1];
    K = a.K;
    if (K < 0 || a.lda < K || a.ldb < N || a.ldc < N) return upir_fail(c, UPIR_EINVAL, "matmul K / leading dims");
    if (kind != UPIR_BODY_MATMUL_F32 && a.workspace &&
        a.workspace_bytes < upir_matmul_workspace_bytes(kind, M, N, K))
      return upir_fail(c, UPIR_EINVAL, "matmul workspace too small");
  }
  if (kind == UPIR_BODY_MATVEC) {
    const upir_matvec_args &a = *(const upir_matvec_args *)body->args;
    if (a.cols < 0 || a.lda < a.cols) return upir_fail(c, UPIR_EINVAL, "matvec cols / lda");
  }
  if (kind == UPIR_BODY_JACOBI5 && ((const upir_jacobi5_args *)body->args)->ld < 1)
    return upir_fail(c, UPIR_EINVAL, "jacobi leading dimension");
  if (kind == UPIR_BODY_FILTER7 && ((const upir_filter7_args *)body->args)->ld < 1)
    return upir_fail(c, UPIR_EINVAL, "filter leading dimension");
  if (has_red && R.result_on_host && c->none) return upir_fail(c, UPIR_ESTATE, "host results need a device");

  lp->ctx = c;
  lp->loop = L;
  lp->sched = S;
  lp->kind = kind;
  lp->args_dev = body->args_are_device_ptrs ? 1 : 0;
  memcpy(lp->args, body->args, asz);
  lp->args_size = asz;
  lp->has_red = has_red;
  lp->red = R;
  for (int d = 0; d < 3; ++d) lp->cnt[d] = cnt[d];
  lp->n = (int64_t)n;
  lp->sum_dtype = sum_dtype;
  lp->key = loop_shape_key(lp);
  return UPIR_OK;
}

extern "C" upir_status upir_loop_parallel(upir_ctx *c, const upir_loop *loop, const upir_sched *sched,
                                          const upir_body *body, const upir_reduction *red, upir_loop_h *out) {
  if (!c) return UPIR_EINVAL;
  if (!loop || !body || !out) return upir_fail(c, UPIR_EINVAL, "loop_parallel: null loop, body or out");
  *out = nullptr;
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "loop_parallel during graph capture");
  upir_loop_obj *lp = new (std::nothrow) upir_loop_obj();
  if (!lp) return upir_fail(c, UPIR_ENOMEM, "loop handle");
  upir_status st = describe_loop(c, loop, sched, body, red, lp);
  if (st) {
    delete lp;
    return st;
  }
  const int32_t kind = lp->kind;
  const bool has_red = lp->has_red;
  lp->part_cap = has_red ? 8192 : 0;
  lp->scratch = (unsigned char *)upir_dalloc(c, scratch_bytes(lp->part_cap));
  if (!lp->scratch) {
    delete lp;
    return upir_fail(c, UPIR_ENOMEM, "reduction scratch");
  }
  if (!c->none) {
    upir_status cs = clear_scratch(c, lp, lp->scratch, lp->part_cap);
    if (cs) {
      free_loop(c, lp);
      return cs;
    }
  }
  if ((kind == UPIR_BODY_MATMUL_BF16 || kind == UPIR_BODY_MATMUL_SPLIT3) &&
      !((const upir_matmul_args *)body->args)->workspace) {
    lp->ws_bytes = upir_matmul_workspace_bytes(kind, lp->cnt[0], lp->cnt[1], ((const upir_matmul_args *)body->args)->K);
    lp->ws = upir_dalloc(c, lp->ws_bytes);
    if (!lp->ws) {
      free_loop(c, lp);
      return upir_fail(c, UPIR_ENOMEM, "matmul workspace (%zu bytes)", lp->ws_bytes);
    }
  }
  c->loops.insert(lp);
  *out = lp;
  return UPIR_OK;
}

extern "C" upir_status upir_loop_free(upir_ctx *c, upir_loop_h lp) {
  if (!c || !lp) return UPIR_EINVAL;
  if (!c->loops.count(lp)) return upir_fail(c, UPIR_EINVAL, "unknown loop handle");
  for (auto &t : c->tasks)
    if (t.loop == lp) return upir_fail(c, UPIR_ESTATE, "loop handle is used by a pending task");
  if (c->pend.on && c->pend.owner == lp) {
    if (c->capturing) return upir_fail(c, UPIR_ESTATE, "loop has a deferred fold in the capture");
    upir_status st = upir::settle(c);
    if (st) return st;
  }
  if (!c->none) (void)hipStreamSynchronize(c->stream);
  c->loops.erase(lp);
  if (c->reduce_loop == lp) c->reduce_loop = nullptr;
  free_loop(c, lp);
  return UPIR_OK;
}

extern "C" upir_status upir_loop_set_result(upir_ctx *c, upir_loop_h lp, void *result) {
  if (!c || !lp || !c->loops.count(lp)) return UPIR_EINVAL;
  if (!lp->has_red) return upir_fail(c, UPIR_ESTATE, "loop has no reduction");
  if (!result) return upir_fail(c, UPIR_EINVAL, "null result");
  lp->red.result = result;
  return UPIR_OK;
}

extern "C" upir_status upir_loop_set_args(upir_ctx *c, upir_loop_h lp, const void *args, size_t sz) {
  if (!c || !lp || !c->loops.count(lp)) return UPIR_EINVAL;
  if (!args || sz != lp->args_size) return upir_fail(c, UPIR_EINVAL, "args size");
  if (lp->kind == UPIR_BODY_SUM && ((const upir_sum_args *)args)->dtype != lp->sum_dtype)
    return upir_fail(c, UPIR_EINVAL, "SUM dtype cannot change");
  memcpy(lp->args, args, sz);
  return UPIR_OK;
}

namespace upir {

uint64_t loop_shape_key(const upir_loop_obj *lp) {
  // FNV-1a over the body kind, trip counts, reduction op and alignment class
  uint64_t h = 1469598103934665603ULL;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xff;
      h *= 1099511628211ULL;
    }
  };
  mix((uint64_t)lp->kind);
  mix((uint64_t)lp->loop.collapse);
  for (int d = 0; d < lp->loop.collapse; ++d) {
    mix((uint64_t)lp->cnt[d]);
    mix((uint64_t)lp->loop.dim[d].step);
    mix((uint64_t)(lp->loop.dim[d].lb & 3));
  }
  mix((uint64_t)(lp->has_red ? lp->red.op : 0));
  if (lp->kind == UPIR_BODY_MATVEC) mix((uint64_t)((const upir_matvec_args *)lp->args)->cols);
  if (is_matmul(lp->kind)) mix((uint64_t)((const upir_matmul_args *)lp->args)->K);
  return h;
}

upir_status resolve_payload(upir_ctx *c, upir_loop_obj *lp, unsigned char *payload) {
  upir_status st = UPIR_OK;
  switch (lp->kind) {
    case UPIR_BODY_AXPY: {
      const upir_axpy_args &a = *(const upir_axpy_args *)lp->args;
      AxpyP p{a.a, nullptr, nullptr};
      const void *x, *y;
      if ((st = xlate(c, lp, a.x, &x)) || (st = xlate(c, lp, a.y, &y))) return st;
      p.x = (const float *)x;
      p.y = (float *)y;
      if (lp->n > 0 && (!p.x || !p.y)) return upir_fail(c, UPIR_EINVAL, "AXPY needs x and y");
      memcpy(payload, &p, sizeof p);
      break;
    }
    case UPIR_BODY_SUM: {
      const upir_sum_args &a = *(const upir_sum_args *)lp->args;
      const void *x;
      if ((st = xlate(c, lp, a.x, &x))) return st;
      if (lp->n > 0 && !x) return upir_fail(c, UPIR_EINVAL, "SUM needs x");
      SumP p{x, a.dtype};
      memcpy(payload, &p, sizeof p);
      break;
    }
    case UPIR_BODY_JACOBI5: {
      const upir_jacobi5_args &a = *(const upir_jacobi5_args *)lp->args;
      const void *s, *d;
      if ((st = xlate(c, lp, a.src, &s)) || (st = xlate(c, lp, a.dst, &d))) return st;
      if (lp->n > 0 && (!s || !d)) return upir_fail(c, UPIR_EINVAL, "JACOBI5 needs src and dst");
      if (lp->n > 0 && s == d) return upir_fail(c, UPIR_EINVAL, "JACOBI5 src and dst must differ");
      JacobiP p{(const float *)s, (float *)d, a.ld};
      memcpy(payload, &p, sizeof p);
      break;
    }
    case UPIR_BODY_FILTER7: {
      const upir_filter7_args &a = *(const upir_filter7_args *)lp->args;
      const void *s, *d, *w;
      if ((st = xlate(c, lp, a.src, &s)) || (st = xlate(c, lp, a.dst, &d)) || (st = xlate(c, lp, a.w, &w))) return st;
      if (lp->n > 0 && (!s || !d || !w)) return upir_fail(c, UPIR_EINVAL, "FILTER7 needs src, dst and w");
      if (lp->n > 0 && s == d) return upir_fail(c, UPIR_EINVAL, "FILTER7 src and dst must differ");
      Filter7P p{(const float *)s, (float *)d, (const float *)w, a.ld};
      memcpy(payload, &p, sizeof p);
      break;
    }
    case UPIR_BODY_MATMUL_F32:
    case UPIR_BODY_MATMUL_BF16:
    case UPIR_BODY_MATMUL_SPLIT3: {
      const upir_matmul_args &a = *(const upir_matmul_args *)lp->args;
      const void *A, *B, *C;
      if ((st = xlate(c, lp, a.A, &A)) || (st = xlate(c, lp, a.B, &B)) || (st = xlate(c, lp, a.C, &C))) return st;
      if (lp->n > 0 && (!A || !B || !C)) return upir_fail(c, UPIR_EINVAL, "MATMUL needs A, B and C");
      MatmulP p{};
      p.A = (const float *)A;
      p.B = (const float *)B;
      p.C = (float *)C;
      p.M = lp->cnt[0];
      p.N = lp->cnt[1];
      p.K = a.K;
      p.lda = a.lda;
      p.ldb = a.ldb;
      p.ldc = a.ldc;
      p.kind = lp->kind;
      uint16_t *ws = (uint16_t *)(a.workspace ? a.workspace : lp->ws);
      if (lp->kind != UPIR_BODY_MATMUL_F32) {
        const int64_t kp = mm_kpad(p.K);
        p.ah = ws;
        p.bh = ws + p.M * kp;
        if (lp->kind == UPIR_BODY_MATMUL_SPLIT3) {
          p.al = p.bh + p.N * kp;
          p.bl = p.al + p.M * kp;
        }
      }
      memcpy(payload, &p, sizeof p);
      break;
    }
    case UPIR_BODY_MATVEC: {
      const upir_matvec_args &a = *(const upir_matvec_args *)lp->args;
      const void *A, *x, *y;
      if ((st = xlate(c, lp, a.A, &A)) || (st = xlate(c, lp, a.x, &x)) || (st = xlate(c, lp, a.y, &y))) return st;
      if (lp->n > 0 && (!A || !x || !y)) return upir_fail(c, UPIR_EINVAL, "MATVEC needs A, x and y");
      MatvecP p{(const float *)A, (const float *)x, (float *)y, a.cols, a.lda};
      memcpy(payload, &p, sizeof p);
      break;
    }
    case UPIR_BODY_OWNER: {
      const void *o;
      if ((st = xlate(c, lp, ((const upir_owner_args *)lp->args)->out, &o))) return st;
      if (lp->n > 0 && !o) return upir_fail(c, UPIR_EINVAL, "OWNER needs out");
      OwnerP p{(int32_t *)o};
      memcpy(payload, &p, sizeof p);
      break;
    }
    case UPIR_BODY_COVER: {
      const void *o;
      if ((st = xlate(c, lp, ((const upir_cover_args *)lp->args)->count, &o))) return st;
      if (lp->n > 0 && !o) return upir_fail(c, UPIR_EINVAL, "COVER needs count");
      CoverP p{(int32_t *)o};
      memcpy(payload, &p, sizeof p);
      break;
    }
    default: return upir_fail(c, UPIR_EINVAL, "body kind");
  }
  return UPIR_OK;
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Library default schedule and geometry for a body (used by AUTO when the
// tuner and the model have nothing to say, and to fill num_teams = 0).
void default_choice(upir_ctx *c, const upir_loop_obj *lp, upir_spmd &sp, upir_sched &sc) {
  const int64_t n = lp->n;
  const int64_t cap = 8LL * c->num_cus;
  sc = upir_sched{};
  sp.target = UPIR_TARGET_GPU;
  sp.num_units = 256;
  switch (lp->kind) {
    case UPIR_BODY_AXPY:
    case UPIR_BODY_COVER:
    case UPIR_BODY_SUM:
      if (lp->loop.collapse == 1) {
        // one 256-unit team per CU at most: fewer, longer streams keep HBM
        // pages open better than many short ones
        sc.policy = UPIR_SCHED_STATIC_CHUNK;
        sc.chunk = 4;
        sp.num_teams = (int32_t)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 16LL * 256), c->num_cus));
      } else {
        sc.policy = UPIR_SCHED_STATIC;
        sp.num_teams = (int32_t)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 8LL * 256), cap));
      }
      break;
    case UPIR_BODY_JACOBI5:
    case UPIR_BODY_FILTER7: {
      // the tallest tile (longest wavefront strips) that still gives every
      // SIMD four wavefronts: at least 4 x CUs tiles of 4 wavefronts each
      // (128-row tiles: Jacobi only)
      sc.policy = UPIR_SCHED_STATIC;
      sc.tile[1] = 256;
      sc.tile[0] = 4;
      const int64_t ct = cdiv(std::max<int64_t>(lp->cnt[1], 1), 256);
      for (int th : {128, 64, 32, 16, 8})
        if ((th < 128 || lp->kind == UPIR_BODY_JACOBI5) &&
            cdiv(std::max<int64_t>(lp->cnt[0], 1), th) * ct >= 4LL * c->num_cus) {
          sc.tile[0] = th;
          break;
        }
      sp.num_teams = 0;  // one tile per team
      break;
    }
    case UPIR_BODY_MATMUL_F32:
    case UPIR_BODY_MATMUL_BF16:
    case UPIR_BODY_MATMUL_SPLIT3: {
      // MFMA tile configurations: bfloat16 and the split's three products
      // 256 x 256 on 4 wavefronts of 128 x 128 each (the split as one product
      // over K' = 3K: 250 us against 355 us for the 8-wavefront tile at
      // 4096^3); 128 x 128 tiles when C has fewer 256 x 256 tiles than half
      // the device's CUs (measured with 256 CUs: 128 x 128 faster at 2048^2,
      // 64 large tiles; 256 x 256 faster at 3072^2, 144 large tiles).
      // float32: 256 x 128 on 8 wavefronts when C has at least one such tile
      // per CU (1.08 against 1.11 ms at 4096^3), else 128 x 128 on 4.
      sc.policy = UPIR_SCHED_STATIC;
      sp.num_teams = 0;
      sp.num_units = 256;
      if (lp->kind == UPIR_BODY_MATMUL_F32) {
        const bool big = cdiv(lp->cnt[0], 256) * cdiv(lp->cnt[1], 128) >= c->num_cus;
        sc.tile[0] = big ? 256 : 128;
        sc.tile[1] = 128;
        sp.num_units = big ? 512 : 256;
        break;
      }
      const bool small = 2 * cdiv(lp->cnt[0], 256) * cdiv(lp->cnt[1], 256) < c->num_cus;
      sc.tile[0] = sc.tile[1] = small ? 128 : 256;
      break;
    }
    case UPIR_BODY_MATVEC:
      sc.policy = UPIR_SCHED_STATIC_CHUNK;
      sc.chunk = 1;
      sp.num_teams = (int32_t)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 4), cap));
      break;
    default:
      sc.policy = UPIR_SCHED_STATIC;
      sp.num_teams = (int32_t)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), cap));
  }
}

static bool parse_runtime_schedule(upir_sched &sc) {
  const char *e = getenv("UPIR_SCHEDULE");
  if (!e) {
    sc.policy = UPIR_SCHED_STATIC;
    return true;
  }
  char name[32] = {0};
  long long ch = 0;
  int got = sscanf(e, "%31[a-z_],%lld", name, &ch);
  if (got < 1) return false;
  if (!strcmp(name, "static")) sc.policy = got == 2 ? UPIR_SCHED_STATIC_CHUNK : UPIR_SCHED_STATIC;
  else if (!strcmp(name, "dynamic")) sc.policy = UPIR_SCHED_DYNAMIC;
  else if (!strcmp(name, "guided")) sc.policy = UPIR_SCHED_GUIDED;
  else return false;
  sc.chunk = got == 2 ? ch : 1;
  if (sc.chunk < 1) return false;
  return true;
}

upir_status resolve_plan(upir_ctx *c, const upir_spmd *spmd_in, upir_loop_obj *lp, Plan &pl) {
  upir_spmd sp{0, 0, UPIR_TARGET_GPU};
  if (spmd_in) sp = *spmd_in;
  if (sp.target == 0) sp.target = UPIR_TARGET_GPU;
  if (sp.target != UPIR_TARGET_GPU) return upir_fail(c, UPIR_EUNSUPPORTED, "only target(gpu) is provided");
  if (sp.num_teams < 0 || sp.num_units < 0 || sp.num_units > 1024)
    return upir_fail(c, UPIR_EINVAL, "num_teams %d / num_units %d", sp.num_teams, sp.num_units);
  upir_sched sc = lp->sched;
  upir_spmd dsp;
  upir_sched dsc;
  default_choice(c, lp, dsp, dsc);
  if (sc.policy == UPIR_SCHED_RUNTIME) {
    upir_sched r{};
    if (!parse_runtime_schedule(r)) return upir_fail(c, UPIR_EINVAL, "UPIR_SCHEDULE is malformed");
    r.distribute = sc.distribute;
    memcpy(r.tile, sc.tile, sizeof r.tile);
    sc = r;
    upir_status st = validate_sched(c, lp->loop, sc, lp->kind);
    if (st) return st;
  } else if (sc.policy == UPIR_SCHED_AUTO) {
    upir_spmd asp = dsp;
    upir_sched asc = dsc;
    auto it = c->tuned.find(lp->key);
    if (it != c->tuned.end()) {
      asp = it->second.spmd;
      asc = it->second.sched;
    } else if (c->model_on) {
      model_pick(c, lp, asp, asc);
    }
    sc = asc;
    if (sp.num_teams == 0) sp.num_teams = asp.num_teams;
    if (sp.num_units == 0) sp.num_units = asp.num_units;
  }
  if (sp.num_units == 0) sp.num_units = dsp.num_units;
  if (lp->kind == UPIR_BODY_MATVEC && (sp.num_units % 64) != 0)
    return upir_fail(c, UPIR_EINVAL, "MATVEC units are wavefronts: num_units must be a multiple of 64");
  LoopK L{};
  L.nd = lp->loop.collapse;
  for (int d = 0; d < 3; ++d) {
    L.lb[d] = d < L.nd ? lp->loop.dim[d].lb : 0;
    L.step[d] = d < L.nd ? lp->loop.dim[d].step : 1;
    L.cnt[d] = lp->cnt[d];
  }
  L.n = lp->n;
  SchedK S{};
  S.policy = sc.policy;
  S.dist = sc.distribute;
  S.chunk = sc.chunk;
  S.tiled = (sc.tile[0] || sc.tile[1] || sc.tile[2]) ? 1 : 0;
  S.ntiles = 0;
  if (S.tiled) {
    S.ntiles = 1;
    for (int d = 0; d < 3; ++d) {
      S.tile[d] = d < L.nd ? sc.tile[d] : 1;
      if (d < L.nd) {
        const int64_t lb = L.lb[d], ub = L.lb[d] + L.cnt[d];
        S.t0[d] = floordiv(lb, S.tile[d]);
        S.nt[d] = L.cnt[d] ? floordiv(ub + S.tile[d] - 1, S.tile[d]) - S.t0[d] : 0;
        S.ntiles *= S.nt[d];
      } else {
        S.t0[d] = 0;
        S.nt[d] = 1;
      }
    }
  }
  int64_t T = sp.num_teams;
  if (S.dist == UPIR_DIST_UNITS) {
    if (T > 1) return upir_fail(c, UPIR_EINVAL, "distribute(units) runs on one team");
    T = 1;
  }
  if (T == 0) {
    if (S.tiled) {
      T = S.policy == UPIR_SCHED_STATIC ? S.ntiles : cdiv(S.ntiles, S.chunk);
      if (is_matmul(lp->kind) || lp->kind == UPIR_BODY_JACOBI5 || lp->kind == UPIR_BODY_FILTER7) T = std::max<int64_t>(T, 1);
    } else {
      T = dsp.num_teams > 0 ? dsp.num_teams : 1;
    }
    T = std::max<int64_t>(1, std::min<int64_t>(T, 1 << 20));
  }
  if (T > (1 << 24)) return upir_fail(c, UPIR_EINVAL, "num_teams too large");
  S.T = (int32_t)T;
  S.U = sp.num_units;
  S.dyn_next = (long long *)(lp->scratch + SCR_DYN);
  S.dyn_exit = (unsigned *)(lp->scratch + SCR_DYNEXIT);
  sp.num_teams = S.T;

  // kernel variant
  int32_t v = V_GENERIC;
  const bool dyn = S.policy == UPIR_SCHED_DYNAMIC || S.policy == UPIR_SCHED_GUIDED;
  if (dyn) {
    v = V_DYNAMIC;
  } else if (lp->kind == UPIR_BODY_MATVEC) {
    v = V_MATVEC_WAVE;
  } else if ((lp->kind == UPIR_BODY_AXPY || lp->kind == UPIR_BODY_COVER ||
              (lp->kind == UPIR_BODY_SUM && lp->sum_dtype == UPIR_DT_F32)) &&
             !S.tiled && S.dist == UPIR_DIST_TEAMS_UNITS && L.nd == 1 && L.step[0] == 1 &&
             ((S.policy == UPIR_SCHED_STATIC_CHUNK && S.chunk == 4) ||
              (S.policy == UPIR_SCHED_STATIC && L.n == 4LL * S.T * S.U))) {
    // the vector path needs 16-byte aligned x (and y) at the first iteration
    unsigned char pay[128];
    if (resolve_payload(c, lp, pay) == UPIR_OK) {
      bool ok = true;
      const int64_t lb = L.lb[0];
      if (lp->kind == UPIR_BODY_AXPY) {
        const AxpyP &p = *(const AxpyP *)pay;
        ok = ((uintptr_t)(p.x + lb) % 16 == 0) && ((uintptr_t)(p.y + lb) % 16 == 0);
      } else if (lp->kind == UPIR_BODY_SUM) {
        const SumP &p = *(const SumP *)pay;
        ok = ((uintptr_t)((const float *)p.x + lb) % 16 == 0);
      } else {
        ok = lb == 0;
      }
      if (ok) v = V_STREAM4;
    }
    c->err.clear();
  } else if (lp->kind == UPIR_BODY_JACOBI5 && S.tiled) {
    unsigned char pay[128];
    if (resolve_payload(c, lp, pay) == UPIR_OK && jacobi_tile_supports(*(const JacobiP *)pay, L, S))
      v = V_JACOBI_TILE;
    c->err.clear();
  } else if (lp->kind == UPIR_BODY_FILTER7 && S.tiled) {
    unsigned char pay[128];
    if (resolve_payload(c, lp, pay) == UPIR_OK && filter7_tile_supports(*(const Filter7P *)pay, L, S))
      v = V_FILTER7_TILE;
    c->err.clear();
  } else if (is_matmul(lp->kind) && S.tiled) {
    unsigned char pay[sizeof(MatmulP) + 16];
    if (resolve_payload(c, lp, pay) == UPIR_OK && matmul_mfma_supports(*(const MatmulP *)pay, L, S))
      v = V_MATMUL_MFMA;
    c->err.clear();
  }
  pl.variant = v;
  pl.L = L;
  pl.S = S;
  pl.spmd = sp;
  pl.sched = sc;
  return UPIR_OK;
}

bool red_is_int(const upir_loop_obj *lp) {
  return lp->kind == UPIR_BODY_SUM && (lp->sum_dtype == UPIR_DT_I32 || lp->sum_dtype == UPIR_DT_I64);
}

// Header zero; reduction slots empty (float: all-ones pattern, int: flag 0).
upir_status clear_scratch(upir_ctx *c, upir_loop_obj *lp, unsigned char *scr, int64_t cap) {
  HIPTRY(c, hipMemsetAsync(scr, 0, SCR_SLOTS, c->stream));
  if (cap > 0)
    HIPTRY(c, hipMemsetAsync(scr + SCR_SLOTS, red_is_int(lp) ? 0 : 0xFF, (size_t)cap * 8 * SLOT_WORDS, c->stream));
  return UPIR_OK;
}

upir_status ensure_scratch(upir_ctx *c, upir_loop_obj *lp, int64_t parts) {
  if (parts <= lp->part_cap) return UPIR_OK;
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "reduction scratch must grow; launch once before capturing");
  if (c->pend.on && c->pend.owner == lp) {
    upir_status st = settle(c);
    if (st) return st;
  }
  HIPTRY(c, hipStreamSynchronize(c->stream));
  // grow geometrically, so a loop launched with ever more teams retires few buffers
  const int64_t cap = std::max<int64_t>(parts, 2 * lp->part_cap);
  unsigned char *ns = (unsigned char *)upir_dalloc(c, scratch_bytes(cap));
  if (!ns) return upir_fail(c, UPIR_ENOMEM, "reduction scratch");
  upir_status st = clear_scratch(c, lp, ns, cap);
  if (st) {
    upir_dfree(c, ns);
    return st;
  }
  // a graph captured earlier still addresses the old block (combiner slots,
  // dynamic-schedule counters): it is kept until finalize, like the
  // outgrown fold buffers
  if (lp->scratch) c->retired.push_back(lp->scratch);
  lp->scratch = ns;
  lp->part_cap = cap;
  return UPIR_OK;
}

upir_status settle(upir_ctx *c) {
  if (!c->pend.on) return UPIR_OK;
  hipError_t e = launch_fold(c->pend.F, c->stream);
  if (e != hipSuccess) return upir_hipfail(c, e, "reduction fold");
  c->pend.on = false;
  c->pend.owner = nullptr;
  return UPIR_OK;
}

// Both fold buffers hold at least `parts` partials. Outgrown buffers are
// kept until finalize: a captured graph may still write them.
static upir_status ensure_fold_bufs(upir_ctx *c, int64_t parts) {
  if (parts <= c->fold_cap) return UPIR_OK;
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "fold buffers must grow; launch once before capturing");
  const int64_t cap = std::max<int64_t>(parts, 1 << 16);
  unsigned long long *nb[2];
  for (int i = 0; i < 2; ++i) {
    nb[i] = (unsigned long long *)upir_dalloc(c, (size_t)cap * 8);
    if (!nb[i]) {
      if (i) upir_dfree(c, nb[0]);
      return upir_fail(c, UPIR_ENOMEM, "fold buffers");
    }
  }
  for (int i = 0; i < 2; ++i) {
    if (c->fold_buf[i]) c->retired.push_back(c->fold_buf[i]);
    c->fold_buf[i] = nb[i];
  }
  c->fold_cap = cap;
  return UPIR_OK;
}

static bool takes_fold(int32_t variant) { return variant != V_MATMUL_MFMA; }

upir_status launch_plan(upir_ctx *c, upir_loop_obj *lp, const Plan &pl, bool for_task) {
  alignas(16) unsigned char pay[sizeof(MatmulP) + 16];
  upir_status st = resolve_payload(c, lp, pay);
  if (st) return st;
  // an async reduction outside the task graph defers its fold
  const bool defer = lp->has_red && lp->red.async && !for_task;
  const int64_t nparts = (int64_t)pl.S.T * ((pl.S.U + 63) / 64);  // one partial per wavefront
  if (defer) {
    st = ensure_fold_bufs(c, nparts);
    if (st) return st;
  }
  RedK R{};
  if (lp->has_red) {
    st = ensure_scratch(c, lp, defer ? 0 : pl.S.T);  // deferred: no combiner slots
    if (st) return st;
    R.op = lp->red.op;
    R.is_int = red_is_int(lp);
    R.init = lp->red.init;
    R.init_i = (long long)lp->red.init;
    R.result = lp->red.result_on_host ? (void *)(lp->scratch + SCR_RESULT) : lp->red.result;
    R.slots = (unsigned long long *)(lp->scratch + SCR_SLOTS);
    R.spin_limit = 1LL << 22;
    if (defer) R.defer = c->fold_buf[c->fold_flip];
  }
  if (c->pend.on) {  // the previous async loop's fold rides on this kernel
    if (takes_fold(pl.variant) && !(lp->n == 0 && !lp->has_red)) {
      R.fold = c->pend.F;
    } else {
      st = settle(c);
      if (st) return st;
    }
  }
  SchedK S = pl.S;
  S.dyn_next = (long long *)(lp->scratch + SCR_DYN);
  S.dyn_exit = (unsigned *)(lp->scratch + SCR_DYNEXIT);
  if (lp->n == 0 && !lp->has_red) return UPIR_OK;  // nothing to run
  hipError_t e = hipSuccess;
  switch (pl.variant) {
    case V_STREAM4: e = launch_stream4(lp->kind, pay, pl.L, S, R, c->stream); break;
    case V_JACOBI_TILE: e = launch_jacobi_tile(*(const JacobiP *)pay, pl.L, S, R, c->stream); break;
    case V_FILTER7_TILE: e = launch_filter7_tile(*(const Filter7P *)pay, pl.L, S, R, c->stream); break;
    case V_MATVEC_WAVE: e = launch_matvec_wave(*(const MatvecP *)pay, pl.L, S, R, c->stream); break;
    case V_MATMUL_MFMA: {
      MatmulP p = *(const MatmulP *)pay;
      p.panel = matmul_wide(p, S) ? 1 : 0;  // the pre-pass writes the layout the tile reads
      if (p.kind != UPIR_BODY_MATMUL_F32) e = launch_bf16_split(p, p.kind == UPIR_BODY_MATMUL_SPLIT3, c->stream);
      if (e == hipSuccess) e = launch_matmul_mfma(p, pl.L, S, c->stream);
      break;
    }
    default: {
      if (is_matmul(lp->kind)) {
        const MatmulP &p = *(const MatmulP *)pay;
        if (p.kind != UPIR_BODY_MATMUL_F32) e = launch_bf16_split(p, p.kind == UPIR_BODY_MATMUL_SPLIT3, c->stream);
        if (e != hipSuccess) break;
      }
      e = launch_generic(lp->kind, pay, pl.L, S, R, c->stream);
    }
  }
  if (e != hipSuccess) return upir_hipfail(c, e, "kernel launch");
  if (R.fold.count > 0) {
    c->pend.on = false;
    c->pend.owner = nullptr;
  }
  if (defer) {
    FoldK F{};
    F.part = R.defer;
    F.count = nparts;
    F.op = R.op;
    F.is_int = R.is_int;
    F.init = R.init;
    F.init_i = R.init_i;
    F.result = R.result;
    c->pend.on = true;
    c->pend.F = F;
    c->pend.owner = lp;
    c->fold_flip ^= 1;
  }
  return UPIR_OK;
}

}  // namespace upir

static upir_status deliver_result(upir_ctx *c, upir_loop_obj *lp) {
  upir_status st = upir::settle(c);
  if (st) return st;
  HIPTRY(c, hipMemcpyAsync(lp->red.result, lp->scratch + SCR_RESULT, 8, hipMemcpyDeviceToHost, c->stream));
  HIPTRY(c, hipStreamSynchronize(c->stream));
  lp->pending = false;
  return UPIR_OK;
}

extern "C" upir_status upir_spmd_launch(upir_ctx *c, const upir_spmd *spmd, const upir_loop_h *loops,
                                        int32_t nloops) {
  if (!c) return UPIR_EINVAL;
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context cannot launch");
  if (nloops < 0 || (nloops > 0 && !loops)) return upir_fail(c, UPIR_EINVAL, "loop list");
  // validate everything before enqueueing anything
  std::vector<Plan> plans(nloops);
  for (int i = 0; i < nloops; ++i) {
    upir_loop_obj *lp = loops[i];
    if (!lp || !c->loops.count(lp)) return upir_fail(c, UPIR_EINVAL, "loop %d: unknown handle", i);
    if (lp->has_red && lp->red.result_on_host && c->capturing)
      return upir_fail(c, UPIR_ESTATE, "host-result reductions cannot be captured");
    upir_status st = resolve_plan(c, spmd, lp, plans[i]);
    if (st) return st;
    alignas(16) unsigned char pay[sizeof(MatmulP) + 16];
    st = resolve_payload(c, lp, pay);
    if (st) return st;
  }
  for (int i = 0; i < nloops; ++i) {
    upir_loop_obj *lp = loops[i];
    upir_status st = launch_plan(c, lp, plans[i], false);
    if (st) return st;
    if (lp->has_red && lp->red.result_on_host) {
      lp->pending = true;
      if (!lp->red.async) {
        st = deliver_result(c, lp);
        if (st) return st;
      }
    }
  }
  return UPIR_OK;
}

extern "C" upir_status upir_reduce_wait(upir_ctx *c, upir_loop_h lp) {
  if (!c || !lp || !c->loops.count(lp)) return UPIR_EINVAL;
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "reduce_wait during graph capture");
  if (!lp->has_red) return upir_fail(c, UPIR_ESTATE, "loop has no reduction");
  if (lp->red.result_on_host) {
    if (!lp->pending) return upir_fail(c, UPIR_ESTATE, "no reduction in flight");
    return deliver_result(c, lp);
  }
  upir_status st = upir::settle(c);
  if (st) return st;
  HIPTRY(c, hipStreamSynchronize(c->stream));
  return UPIR_OK;
}

extern "C" upir_status upir_reduce(upir_ctx *c, int32_t op, int32_t dtype, const void *dev_in, int64_t n,
                                   const upir_spmd *spmd, const upir_sched *sched, upir_reduction *red) {
  if (!c) return UPIR_EINVAL;
  if (!red || !red->result) return upir_fail(c, UPIR_EINVAL, "reduce: result");
  if (op < UPIR_RED_SUM || op > UPIR_RED_MIN) return upir_fail(c, UPIR_EINVAL, "reduce: op");
  if (dtype < UPIR_DT_F32 || dtype > UPIR_DT_I64) return upir_fail(c, UPIR_EINVAL, "reduce: dtype");
  if (n < 0 || (n > 0 && !dev_in)) return upir_fail(c, UPIR_EINVAL, "reduce: input");
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
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
  upir_loop_h lp = nullptr;
  upir_status st = upir_loop_parallel(c, &L, &s, &b, &r, &lp);
  if (st) return st;
  st = upir_spmd_launch(c, spmd, &lp, 1);
  if (!red->result_on_host && st == UPIR_OK) {
    // the handle's scratch must outlive the kernel
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = upir_hipfail(c, e, "reduce");
  }
  upir_loop_free(c, lp);
  return st;
}

extern "C" upir_status upir_loop_resolve(upir_ctx *c, const upir_spmd *spmd, upir_loop_h lp, upir_spmd *sp_out,
                                         upir_sched *sc_out, int32_t *variant_out) {
  if (!c || !lp || !c->loops.count(lp)) return UPIR_EINVAL;
  Plan pl;
  upir_status st = resolve_plan(c, spmd, lp, pl);
  if (st) return st;
  if (sp_out) *sp_out = pl.spmd;
  if (sc_out) *sc_out = pl.sched;
  if (variant_out) *variant_out = pl.variant;
  return UPIR_OK;
}

// ------------------------------------------------------------------ graphs
extern "C" upir_status upir_graph_begin(upir_ctx *c) {
  if (!c) return UPIR_EINVAL;
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "already capturing");
  upir_status st = upir::settle(c);  // folds pending from eager launches stay outside the graph
  if (st) return st;
  HIPTRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
  c->capturing = true;
  return UPIR_OK;
}

extern "C" upir_status upir_graph_end(upir_ctx *c, upir_graph_h *out) {
  if (!c || !out) return UPIR_EINVAL;
  if (!c->capturing) return upir_fail(c, UPIR_ESTATE, "not capturing");
  // the graph's last deferred fold is part of the graph
  const upir_status fs = upir::settle(c);
  c->capturing = false;
  upir_graph_obj *g = new upir_graph_obj();
  hipError_t e = hipStreamEndCapture(c->stream, &g->graph);
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return upir_hipfail(c, e, "graph capture");
  }
  if (fs) {
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return fs;
  }
  c->graphs.insert(g);
  *out = g;
  return UPIR_OK;
}

extern "C" upir_status upir_graph_launch(upir_ctx *c, upir_graph_h g) {
  if (!c || !g || !c->graphs.count(g)) return UPIR_EINVAL;
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "graph launch during capture");
  upir_status st = upir::settle(c);  // the graph reuses the fold buffers
  if (st) return st;
  HIPTRY(c, hipGraphLaunch(g->exec, c->stream));
  return UPIR_OK;
}

extern "C" upir_status upir_graph_destroy(upir_ctx *c, upir_graph_h g) {
  if (!c || !g || !c->graphs.count(g)) return UPIR_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  for (void *p : g->owned) upir_dfree(c, p);
  c->graphs.erase(g);
  delete g;
  return UPIR_OK;
}
