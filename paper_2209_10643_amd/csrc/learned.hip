// Schedule selection for schedule(auto): exhaustive tuner and a learned
// cost model.
//
// The paper's loop_parallel grammar (sec. 3.2) offers schedule(auto), which
// leaves the schedule to the implementation. Here AUTO resolves, in order,
// to the tuner's measured best for the loop's shape, to the cost model's
// choice, and to the library default.
//
//  * Tuner: every candidate (teams, units, chunk, tile) of a loop is timed
//    with HIP events on scratch copies of the loop's read-write outputs; one
//    row per (loop, candidate) goes into the context's timing table.
//  * Cost model: an MLP 32 -> 64 -> 64 -> 1 (float32) predicts log2(time in
//    microseconds) from 32 features of (loop, candidate). It is trained on
//    the timing table by this file's own kernels: forward, backward (per-row
//    deltas, then one thread per parameter summing rows in order) and Adam.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "runtime_internal.h"

using namespace upir;

namespace {

constexpr int F = 32, H1 = 64, H2 = 64;
constexpr int O_W1 = 0, O_B1 = O_W1 + H1 * F, O_W2 = O_B1 + H1, O_B2 = O_W2 + H2 * H1, O_W3 = O_B2 + H2,
              O_B3 = O_W3 + H2, NP = O_B3 + 1;
static_assert(NP == UPIR_MLP_PARAMS, "parameter count");

// ------------------------------------------------------------------ kernels
// Forward pass, one row per thread, parameters staged in LDS. Optionally
// keeps the pre-activations z1, z2 of every row for the backward pass.
__global__ void __launch_bounds__(256) k_mlp_fwd(const float *__restrict__ X, int64_t n, const float *__restrict__ P,
                                                 float *__restrict__ Y, float *__restrict__ Z1, float *__restrict__ Z2) {
  __shared__ float sp[NP];
  for (int i = threadIdx.x; i < NP; i += blockDim.x) sp[i] = P[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float x[F], h1[H1];
  for (int k = 0; k < F; ++k) x[k] = X[r * F + k];
  for (int j = 0; j < H1; ++j) {
    float z = sp[O_B1 + j];
    for (int k = 0; k < F; ++k) z = __builtin_fmaf(sp[O_W1 + j * F + k], x[k], z);
    if (Z1) Z1[r * H1 + j] = z;
    h1[j] = z > 0.0f ? z : 0.0f;
  }
  float y = sp[O_B3];
  for (int j = 0; j < H2; ++j) {
    float z = sp[O_B2 + j];
    for (int k = 0; k < H1; ++k) z = __builtin_fmaf(sp[O_W2 + j * H1 + k], h1[k], z);
    if (Z2) Z2[r * H2 + j] = z;
    y = __builtin_fmaf(sp[O_W3 + j], z > 0.0f ? z : 0.0f, y);
  }
  Y[r] = y;
}

// Per-row deltas: dy = 2 (y - t) / B, dz2 = dy W3 * [z2 > 0],
// dz1 = (dz2 W2) * [z1 > 0]; also the row's squared error.
__global__ void __launch_bounds__(256) k_mlp_bwd_rows(const float *__restrict__ Y, const float *__restrict__ T,
                                                      int64_t B, const float *__restrict__ P,
                                                      const float *__restrict__ Z1, const float *__restrict__ Z2,
                                                      float *__restrict__ DY, float *__restrict__ DZ1,
                                                      float *__restrict__ DZ2, float *__restrict__ SE) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B) return;
  const float d = Y[r] - T[r];
  SE[r] = d * d;
  const float dy = 2.0f * d / (float)B;
  DY[r] = dy;
  float dz2[H2];
  for (int j = 0; j < H2; ++j) {
    dz2[j] = Z2[r * H2 + j] > 0.0f ? dy * P[O_W3 + j] : 0.0f;
    DZ2[r * H2 + j] = dz2[j];
  }
  for (int k = 0; k < H1; ++k) {
    float s = 0.0f;
    for (int j = 0; j < H2; ++j) s = __builtin_fmaf(dz2[j], P[O_W2 + j * H1 + k], s);
    DZ1[r * H1 + k] = Z1[r * H1 + k] > 0.0f ? s : 0.0f;
  }
}

// One thread per parameter (+1 for the loss): sums its gradient over the
// batch rows in row order.
__global__ void __launch_bounds__(256) k_mlp_grad(const float *__restrict__ X, int64_t B, const float *__restrict__ Z1,
                                                  const float *__restrict__ Z2, const float *__restrict__ DY,
                                                  const float *__restrict__ DZ1, const float *__restrict__ DZ2,
                                                  const float *__restrict__ SE, float *__restrict__ G,
                                                  float *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > NP) return;
  float s = 0.0f;
  if (p == NP) {
    for (int64_t r = 0; r < B; ++r) s += SE[r];
    *loss = s / (float)B;
    return;
  }
  if (p < O_B1) {  // W1[j][k] = sum_r dz1[r][j] x[r][k]
    const int j = p / F, k = p % F;
    for (int64_t r = 0; r < B; ++r) s = __builtin_fmaf(DZ1[r * H1 + j], X[r * F + k], s);
  } else if (p < O_W2) {
    const int j = p - O_B1;
    for (int64_t r = 0; r < B; ++r) s += DZ1[r * H1 + j];
  } else if (p < O_B2) {  // W2[j][k] = sum_r dz2[r][j] h1[r][k]
    const int q = p - O_W2, j = q / H1, k = q % H1;
    for (int64_t r = 0; r < B; ++r) {
      const float z = Z1[r * H1 + k];
      s = __builtin_fmaf(DZ2[r * H2 + j], z > 0.0f ? z : 0.0f, s);
    }
  } else if (p < O_W3) {
    const int j = p - O_B2;
    for (int64_t r = 0; r < B; ++r) s += DZ2[r * H2 + j];
  } else if (p < O_B3) {  // W3[j] = sum_r dy[r] h2[r][j]
    const int j = p - O_W3;
    for (int64_t r = 0; r < B; ++r) {
      const float z = Z2[r * H2 + j];
      s = __builtin_fmaf(DY[r], z > 0.0f ? z : 0.0f, s);
    }
  } else {
    for (int64_t r = 0; r < B; ++r) s += DY[r];
  }
  G[p] = s;
}

// Adam with bias correction (Kingma & Ba 2015).
__global__ void __launch_bounds__(256) k_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ M,
                                              float *__restrict__ V, float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float g = G[p];
  const float m = b1 * M[p] + (1.0f - b1) * g;
  const float v = b2 * V[p] + (1.0f - b2) * g * g;
  M[p] = m;
  V[p] = v;
  const float mh = m / c1, vh = v / c2;
  P[p] = P[p] - lr * mh / (sqrtf(vh) + eps);
}

// Row gather for minibatches: dst[i] = src[idx[i]] (rows of `w` floats).
__global__ void k_gather(const float *__restrict__ src, const int32_t *__restrict__ idx, int64_t n, int w,
                         float *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * w) return;
  const int64_t i = e / w, k = e % w;
  dst[e] = src[(int64_t)idx[i] * w + k];
}

uint64_t mix64(uint64_t z) {  // SplitMix64 finalizer (Steele, Lea, Flood 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
uint64_t hash_at(uint64_t seed, uint64_t stream, uint64_t i) {
  const uint64_t G = 0x9E3779B97F4A7C15ULL;
  return mix64(mix64(seed + stream * G) + (i + 1) * G);
}

}  // namespace

struct ModelState {
  float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr;  // device, NP each
  int64_t step = 0;
  uint64_t seed = 0;
  int64_t epochs = 0;
  // work buffers for batches of up to `cap` rows
  int64_t cap = 0;
  float *X = nullptr, *T = nullptr, *Y = nullptr, *Z1 = nullptr, *Z2 = nullptr, *DY = nullptr, *DZ1 = nullptr,
        *DZ2 = nullptr, *SE = nullptr, *loss = nullptr;
};

void upir_model_free(upir_ctx *c) {
  ModelState *m = c->model;
  if (!m) return;
  for (float *p : {m->P, m->M, m->V, m->G, m->X, m->T, m->Y, m->Z1, m->Z2, m->DY, m->DZ1, m->DZ2, m->SE, m->loss})
    upir_dfree(c, p);
  delete m;
  c->model = nullptr;
}

#define HIPTRY(c, expr)                                      \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return upir_hipfail(c, e_, #expr); \
  } while (0)

static upir_status model_buffers(upir_ctx *c, int64_t rows) {
  ModelState *m = c->model;
  if (rows <= m->cap) return UPIR_OK;
  for (float **p : {&m->X, &m->T, &m->Y, &m->Z1, &m->Z2, &m->DY, &m->DZ1, &m->DZ2, &m->SE}) {
    upir_dfree(c, *p);
    *p = nullptr;
  }
  const size_t r = (size_t)rows;
  m->X = (float *)upir_dalloc(c, r * F * 4);
  m->T = (float *)upir_dalloc(c, r * 4);
  m->Y = (float *)upir_dalloc(c, r * 4);
  m->Z1 = (float *)upir_dalloc(c, r * H1 * 4);
  m->Z2 = (float *)upir_dalloc(c, r * H2 * 4);
  m->DY = (float *)upir_dalloc(c, r * 4);
  m->DZ1 = (float *)upir_dalloc(c, r * H1 * 4);
  m->DZ2 = (float *)upir_dalloc(c, r * H2 * 4);
  m->SE = (float *)upir_dalloc(c, r * 4);
  if (!m->X || !m->T || !m->Y || !m->Z1 || !m->Z2 || !m->DY || !m->DZ1 || !m->DZ2 || !m->SE)
    return upir_fail(c, UPIR_ENOMEM, "model work buffers");
  m->cap = rows;
  return UPIR_OK;
}

static upir_status need_model(upir_ctx *c) {
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
  if (!c->model) return upir_fail(c, UPIR_ESTATE, "no model: call upir_model_init or upir_model_load");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "model calls during graph capture");
  return UPIR_OK;
}

extern "C" upir_status upir_model_init(upir_ctx *c, uint64_t seed) {
  if (!c) return UPIR_EINVAL;
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
  upir_model_free(c);
  ModelState *m = new ModelState();
  c->model = m;
  m->seed = seed;
  m->P = (float *)upir_dalloc(c, NP * 4);
  m->M = (float *)upir_dalloc(c, NP * 4);
  m->V = (float *)upir_dalloc(c, NP * 4);
  m->G = (float *)upir_dalloc(c, NP * 4);
  m->loss = (float *)upir_dalloc(c, 64);
  if (!m->P || !m->M || !m->V || !m->G || !m->loss) {
    upir_model_free(c);
    return upir_fail(c, UPIR_ENOMEM, "model parameters");
  }
  // Kaiming-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)), zero biases
  std::vector<float> h(NP, 0.0f);
  auto fill = [&](int off, int count, int fan_in, uint64_t stream) {
    const double bound = sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) {
      const int64_t k = (int64_t)(hash_at(seed, stream, i) >> 40) - (1 << 23);  // [-2^23, 2^23)
      h[off + i] = (float)(bound * (double)k * 0x1p-23);
    }
  };
  fill(O_W1, H1 * F, F, 1);
  fill(O_W2, H2 * H1, H1, 2);
  fill(O_W3, H2, H2, 3);
  std::vector<float> zero(NP, 0.0f);
  HIPTRY(c, hipMemcpyAsync(m->P, h.data(), NP * 4, hipMemcpyHostToDevice, c->stream));
  HIPTRY(c, hipMemcpyAsync(m->M, zero.data(), NP * 4, hipMemcpyHostToDevice, c->stream));
  HIPTRY(c, hipMemcpyAsync(m->V, zero.data(), NP * 4, hipMemcpyHostToDevice, c->stream));
  HIPTRY(c, hipStreamSynchronize(c->stream));
  m->step = 0;
  return UPIR_OK;
}

extern "C" upir_status upir_model_set_params(upir_ctx *c, const float *host) {
  if (!c || !host) return UPIR_EINVAL;
  upir_status st = need_model(c);
  if (st) return st;
  HIPTRY(c, hipMemcpyAsync(c->model->P, host, NP * 4, hipMemcpyHostToDevice, c->stream));
  std::vector<float> zero(NP, 0.0f);
  HIPTRY(c, hipMemcpyAsync(c->model->M, zero.data(), NP * 4, hipMemcpyHostToDevice, c->stream));
  HIPTRY(c, hipMemcpyAsync(c->model->V, zero.data(), NP * 4, hipMemcpyHostToDevice, c->stream));
  HIPTRY(c, hipStreamSynchronize(c->stream));
  c->model->step = 0;
  return UPIR_OK;
}

extern "C" upir_status upir_model_get_params(upir_ctx *c, float *host) {
  if (!c || !host) return UPIR_EINVAL;
  upir_status st = need_model(c);
  if (st) return st;
  HIPTRY(c, hipMemcpyAsync(host, c->model->P, NP * 4, hipMemcpyDeviceToHost, c->stream));
  HIPTRY(c, hipStreamSynchronize(c->stream));
  return UPIR_OK;
}

static hipError_t fwd_launch(upir_ctx *c, const float *X, int64_t n, float *Y, float *Z1, float *Z2) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, X, n, c->model->P, Y, Z1,
                     Z2);
  return hipGetLastError();
}

extern "C" upir_status upir_model_forward(upir_ctx *c, const float *dev_x, int64_t n, float *dev_y) {
  if (!c) return UPIR_EINVAL;
  upir_status st = need_model(c);
  if (st) return st;
  if (n < 0 || (n > 0 && (!dev_x || !dev_y))) return upir_fail(c, UPIR_EINVAL, "model_forward arguments");
  HIPTRY(c, fwd_launch(c, dev_x, n, dev_y, nullptr, nullptr));
  return UPIR_OK;
}

// One optimisation step on rows already on the device (X: n x 32, T: n).
static upir_status step_dev(upir_ctx *c, const float *X, const float *T, int64_t n, float lr, bool adam,
                            float *grad_out, float *loss_out) {
  ModelState *m = c->model;
  upir_status st = model_buffers(c, n);
  if (st) return st;
  HIPTRY(c, fwd_launch(c, X, n, m->Y, m->Z1, m->Z2));
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_mlp_bwd_rows, dim3(g), dim3(256), 0, c->stream, m->Y, T, n, m->P, m->Z1, m->Z2, m->DY, m->DZ1,
                     m->DZ2, m->SE);
  hipLaunchKernelGGL(k_mlp_grad, dim3((NP + 1 + 255) / 256), dim3(256), 0, c->stream, X, n, m->Z1, m->Z2, m->DY,
                     m->DZ1, m->DZ2, m->SE, m->G, m->loss);
  HIPTRY(c, hipGetLastError());
  if (grad_out) HIPTRY(c, hipMemcpyAsync(grad_out, m->G, NP * 4, hipMemcpyDeviceToDevice, c->stream));
  if (adam) {
    m->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - pow(0.9, (double)m->step)), c2 = (float)(1.0 - pow(0.999, (double)m->step));
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, c->stream, m->P, m->G, m->M, m->V, lr, b1, b2,
                       1e-8f, c1, c2);
    HIPTRY(c, hipGetLastError());
  }
  if (loss_out) {
    HIPTRY(c, hipMemcpyAsync(loss_out, m->loss, 4, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
  }
  return UPIR_OK;
}

extern "C" upir_status upir_model_step(upir_ctx *c, const float *dev_x, const float *dev_t, int64_t n, float lr,
                                       int32_t adam, float *dev_grad, float *loss_out) {
  if (!c) return UPIR_EINVAL;
  upir_status st = need_model(c);
  if (st) return st;
  if (n <= 0 || !dev_x || !dev_t) return upir_fail(c, UPIR_EINVAL, "model_step arguments");
  return step_dev(c, dev_x, dev_t, n, lr, adam != 0, dev_grad, loss_out);
}

// ------------------------------------------------------------ timing table
extern "C" upir_status upir_tune_db_size(upir_ctx *c, int64_t *rows) {
  if (!c || !rows) return UPIR_EINVAL;
  *rows = (int64_t)c->db.size();
  return UPIR_OK;
}

extern "C" upir_status upir_tune_db_row(upir_ctx *c, int64_t row, float *feat, float *log2_us, int64_t *key) {
  if (!c) return UPIR_EINVAL;
  if (row < 0 || row >= (int64_t)c->db.size()) return upir_fail(c, UPIR_EINVAL, "row %lld", (long long)row);
  const TuneRow &r = c->db[row];
  if (feat) memcpy(feat, r.feat, sizeof r.feat);
  if (log2_us) *log2_us = r.log2_us;
  if (key) *key = r.loop_key;
  return UPIR_OK;
}

extern "C" upir_status upir_tune_db_save(upir_ctx *c, const char *path) {
  if (!c || !path) return UPIR_EINVAL;
  FILE *f = fopen(path, "w");
  if (!f) return upir_fail(c, UPIR_EINVAL, "cannot write %s", path);
  fprintf(f, "# upir timing table v1: loop_key log2_us f0..f31\n");
  for (const TuneRow &r : c->db) {
    fprintf(f, "%lld %.9g", (long long)r.loop_key, r.log2_us);
    for (int i = 0; i < F; ++i) fprintf(f, " %.9g", r.feat[i]);
    fputc('\n', f);
  }
  fclose(f);
  return UPIR_OK;
}

extern "C" upir_status upir_tune_db_load(upir_ctx *c, const char *path) {
  if (!c || !path) return UPIR_EINVAL;
  FILE *f = fopen(path, "r");
  if (!f) return upir_fail(c, UPIR_EINVAL, "cannot read %s", path);
  char line[4096];
  std::vector<TuneRow> rows;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    TuneRow r{};
    long long key;
    int used = 0, off = 0;
    if (sscanf(line, "%lld %f%n", &key, &r.log2_us, &used) != 2) {
      fclose(f);
      return upir_fail(c, UPIR_EINVAL, "malformed row in %s", path);
    }
    off = used;
    for (int i = 0; i < F; ++i) {
      if (sscanf(line + off, "%f%n", &r.feat[i], &used) != 1) {
        fclose(f);
        return upir_fail(c, UPIR_EINVAL, "short row in %s", path);
      }
      off += used;
    }
    r.loop_key = key;
    rows.push_back(r);
  }
  fclose(f);
  c->db.insert(c->db.end(), rows.begin(), rows.end());
  return UPIR_OK;
}

// ----------------------------------------------------------------- training
extern "C" upir_status upir_model_train(upir_ctx *c, int32_t epochs, int32_t batch, float lr, int32_t holdout_mod,
                                        float *train_mse, float *holdout_mse) {
  if (!c) return UPIR_EINVAL;
  upir_status st = need_model(c);
  if (st) return st;
  if (epochs < 0 || batch < 1 || batch > 65536) return upir_fail(c, UPIR_EINVAL, "epochs / batch");
  std::vector<int32_t> train, hold;
  for (int32_t i = 0; i < (int32_t)c->db.size(); ++i) {
    const uint64_t k = (uint64_t)c->db[i].loop_key;
    if (holdout_mod >= 0 && (int32_t)(k % 5) == holdout_mod)
      hold.push_back(i);
    else
      train.push_back(i);
  }
  if (train.empty()) return upir_fail(c, UPIR_ESTATE, "no training rows");
  // the whole table on the device once
  const size_t nrow = c->db.size();
  std::vector<float> hx(nrow * F), ht(nrow);
  for (size_t i = 0; i < nrow; ++i) {
    memcpy(&hx[i * F], c->db[i].feat, F * 4);
    ht[i] = c->db[i].log2_us;
  }
  float *dX = (float *)upir_dalloc(c, nrow * F * 4), *dT = (float *)upir_dalloc(c, nrow * 4);
  int32_t *dIdx = (int32_t *)upir_dalloc(c, std::max(train.size(), hold.size()) * 4);
  float *bX = (float *)upir_dalloc(c, (size_t)batch * F * 4), *bT = (float *)upir_dalloc(c, (size_t)batch * 4);
  auto cleanup = [&]() {
    upir_dfree(c, dX);
    upir_dfree(c, dT);
    upir_dfree(c, dIdx);
    upir_dfree(c, bX);
    upir_dfree(c, bT);
  };
  if (!dX || !dT || !dIdx || !bX || !bT) {
    cleanup();
    return upir_fail(c, UPIR_ENOMEM, "training buffers");
  }
  hipError_t e = hipMemcpyAsync(dX, hx.data(), nrow * F * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dT, ht.data(), nrow * 4, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) {
    cleanup();
    return upir_hipfail(c, e, "training copy");
  }
  std::vector<int32_t> order = train;
  for (int32_t ep = 0; ep < epochs && st == UPIR_OK; ++ep) {
    // Fisher-Yates shuffle driven by SplitMix64 (seed, epoch)
    for (size_t i = order.size(); i > 1; --i) {
      const size_t j = (size_t)(hash_at(c->model->seed, 1000 + (uint64_t)(c->model->epochs + ep), i) % i);
      std::swap(order[i - 1], order[j]);
    }
    e = hipMemcpyAsync(dIdx, order.data(), order.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
      st = upir_hipfail(c, e, "index copy");
      break;
    }
    for (size_t b0 = 0; b0 < order.size(); b0 += batch) {
      const int64_t nb = (int64_t)std::min<size_t>(batch, order.size() - b0);
      hipLaunchKernelGGL(k_gather, dim3((unsigned)((nb * F + 255) / 256)), dim3(256), 0, c->stream, dX, dIdx + b0, nb,
                         F, bX);
      hipLaunchKernelGGL(k_gather, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, c->stream, dT, dIdx + b0, nb, 1,
                         bT);
      st = step_dev(c, bX, bT, nb, lr, true, nullptr, nullptr);
      if (st) break;
    }
    // keep the index buffer alive until this epoch's kernels have read it
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess && st == UPIR_OK) st = upir_hipfail(c, e, "training epoch");
  }
  c->model->epochs += epochs;
  // final errors over the train / holdout rows
  auto mse = [&](const std::vector<int32_t> &rows, float *out) -> upir_status {
    if (!out) return UPIR_OK;
    if (rows.empty()) {
      *out = NAN;
      return UPIR_OK;
    }
    float *dY = (float *)upir_dalloc(c, rows.size() * 4);
    float *gX = (float *)upir_dalloc(c, rows.size() * F * 4);
    if (!dY || !gX) {
      upir_dfree(c, dY);
      upir_dfree(c, gX);
      return upir_fail(c, UPIR_ENOMEM, "evaluation buffers");
    }
    hipError_t e2 = hipMemcpyAsync(dIdx, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, c->stream);
    const int64_t n = (int64_t)rows.size();
    if (e2 == hipSuccess) {
      hipLaunchKernelGGL(k_gather, dim3((unsigned)((n * F + 255) / 256)), dim3(256), 0, c->stream, dX, dIdx, n, F, gX);
      e2 = fwd_launch(c, gX, n, dY, nullptr, nullptr);
    }
    std::vector<float> y(n);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(y.data(), dY, n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
    upir_dfree(c, dY);
    upir_dfree(c, gX);
    if (e2 != hipSuccess) return upir_hipfail(c, e2, "evaluation");
    double s = 0;
    for (int64_t i = 0; i < n; ++i) {
      const double d = (double)y[i] - ht[rows[i]];
      s += d * d;
    }
    *out = (float)(s / n);
    return UPIR_OK;
  };
  if (st == UPIR_OK) st = mse(train, train_mse);
  if (st == UPIR_OK) st = mse(hold, holdout_mse);
  cleanup();
  return st;
}

extern "C" upir_status upir_model_enable(upir_ctx *c, int32_t on) {
  if (!c) return UPIR_EINVAL;
  if (on && !c->model) return upir_fail(c, UPIR_ESTATE, "no model");
  c->model_on = on != 0;
  return UPIR_OK;
}

extern "C" upir_status upir_model_save(upir_ctx *c, const char *path) {
  if (!c || !path) return UPIR_EINVAL;
  upir_status st = need_model(c);
  if (st) return st;
  std::vector<float> p(NP);
  st = upir_model_get_params(c, p.data());
  if (st) return st;
  uint64_t sum = 1469598103934665603ULL;
  for (float v : p) {
    uint32_t b;
    memcpy(&b, &v, 4);
    sum = (sum ^ b) * 1099511628211ULL;
  }
  FILE *f = fopen(path, "wb");
  if (!f) return upir_fail(c, UPIR_EINVAL, "cannot write %s", path);
  const int32_t hdr[4] = {0x52495055 /* "UPIR" */, F, H1, H2};
  const int64_t meta[3] = {(int64_t)c->model->seed, c->model->epochs, (int64_t)sum};
  bool ok = fwrite(hdr, sizeof hdr, 1, f) == 1 && fwrite(meta, sizeof meta, 1, f) == 1 &&
            fwrite(p.data(), 4, NP, f) == (size_t)NP;
  fclose(f);
  return ok ? UPIR_OK : upir_fail(c, UPIR_EINVAL, "short write %s", path);
}

extern "C" upir_status upir_model_load(upir_ctx *c, const char *path) {
  if (!c || !path) return UPIR_EINVAL;
  FILE *f = fopen(path, "rb");
  if (!f) return upir_fail(c, UPIR_EINVAL, "cannot read %s", path);
  int32_t hdr[4];
  int64_t meta[3];
  std::vector<float> p(NP);
  bool ok = fread(hdr, sizeof hdr, 1, f) == 1 && fread(meta, sizeof meta, 1, f) == 1 &&
            fread(p.data(), 4, NP, f) == (size_t)NP;
  fclose(f);
  if (!ok || hdr[0] != 0x52495055 || hdr[1] != F || hdr[2] != H1 || hdr[3] != H2)
    return upir_fail(c, UPIR_EINVAL, "%s is not a model file of this shape", path);
  uint64_t sum = 1469598103934665603ULL;
  for (float v : p) {
    uint32_t b;
    memcpy(&b, &v, 4);
    sum = (sum ^ b) * 1099511628211ULL;
  }
  if ((int64_t)sum != meta[2]) return upir_fail(c, UPIR_EINVAL, "%s: checksum mismatch", path);
  upir_status st = upir_model_init(c, (uint64_t)meta[0]);
  if (st) return st;
  st = upir_model_set_params(c, p.data());
  if (st == UPIR_OK) c->model->epochs = meta[1];
  return st;
}

// ----------------------------------------------------- candidates, features
namespace upir {

static double lg(double v) { return v > 0 ? log2(v) : 0.0; }

struct Cand {
  upir_spmd sp;
  upir_sched sc;
};

static bool is_mm(int32_t k) { return k >= UPIR_BODY_MATMUL_F32 && k <= UPIR_BODY_MATMUL_SPLIT3; }

// Candidate schedules of a loop. Candidate 0 is always the library default,
// so the table records what the default costs next to every alternative.
static std::vector<Cand> candidates(upir_ctx *c, const upir_loop_obj *lp) {
  std::vector<Cand> v;
  const int64_t n = lp->n;
  {
    Cand d{};
    default_choice(c, lp, d.sp, d.sc);
    v.push_back(d);
  }
  auto add = [&](int32_t T, int32_t U, int32_t pol, int64_t chunk, int t0 = 0, int t1 = 0) {
    Cand k{};
    k.sp = upir_spmd{T, U, UPIR_TARGET_GPU};
    k.sc.policy = pol;
    k.sc.chunk = chunk;
    k.sc.distribute = UPIR_DIST_TEAMS_UNITS;
    k.sc.tile[0] = t0;
    k.sc.tile[1] = t1;
    v.push_back(k);
  };
  const int64_t capT = 1 << 20;
  auto teams = [&](int64_t work, int64_t per) {
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(capT, (work + per - 1) / per));
  };
  switch (lp->kind) {
    case UPIR_BODY_AXPY:
    case UPIR_BODY_COVER:
    case UPIR_BODY_SUM:
      if (lp->loop.collapse == 1 && (lp->kind != UPIR_BODY_SUM || lp->sum_dtype == UPIR_DT_F32)) {
        for (int32_t U : {64, 256, 1024})
          for (int64_t per : {4, 16, 64, 256}) add(teams(n, U * per), U, UPIR_SCHED_STATIC_CHUNK, 4);
        for (int32_t U : {256, 512})  // one team per CU
          add((int32_t)std::min<int64_t>(c->num_cus, teams(n, U * 4)), U, UPIR_SCHED_STATIC_CHUNK, 4);
      } else {
        for (int32_t U : {64, 256, 1024})
          for (int64_t per : {1, 8, 64}) add(teams(n, U * per), U, UPIR_SCHED_STATIC, 0);
      }
      break;
    case UPIR_BODY_JACOBI5:
    case UPIR_BODY_FILTER7:
      for (int th : {8, 16, 32, 64, 128})
        for (int32_t U : {64, 128, 256, 512})
          if (U <= th * 64 && (th < 128 || lp->kind == UPIR_BODY_JACOBI5)) add(0, U, UPIR_SCHED_STATIC, 0, th, 256);
      break;
    case UPIR_BODY_MATVEC:
      for (int32_t U : {64, 256, 1024})
        for (int64_t rpw : {1, 4, 16}) add(teams(n, (U / 64) * rpw), U, UPIR_SCHED_STATIC_CHUNK, 1);
      break;
    case UPIR_BODY_MATMUL_F32:
      add(0, 256, UPIR_SCHED_STATIC, 0, 128, 128);
      add(0, 512, UPIR_SCHED_STATIC, 0, 256, 128);
      break;
    case UPIR_BODY_MATMUL_BF16:
    case UPIR_BODY_MATMUL_SPLIT3:
      add(0, 256, UPIR_SCHED_STATIC, 0, 128, 128);
      add(0, 256, UPIR_SCHED_STATIC, 0, 256, 256);
      add(0, 512, UPIR_SCHED_STATIC, 0, 256, 256);
      break;
    default:
      for (int32_t U : {64, 256}) add(teams(n, U * 4), U, UPIR_SCHED_STATIC, 0);
  }
  return v;
}

int candidate_count(upir_ctx *c, const upir_loop_obj *lp) { return (int)candidates(c, lp).size(); }

bool candidate_at(upir_ctx *c, const upir_loop_obj *lp, int idx, upir_spmd &sp, upir_sched &sc) {
  auto v = candidates(c, lp);
  if (idx < 0 || idx >= (int)v.size()) return false;
  sp = v[idx].sp;
  sc = v[idx].sc;
  return true;
}

// 32 features of (loop, candidate). Sizes enter as log2 / 32.
static void features(const upir_loop_obj *lp, const Cand &k, float f[32]) {
  for (int i = 0; i < 32; ++i) f[i] = 0.0f;
  const int kind = lp->kind;
  const int cls = kind == UPIR_BODY_AXPY || kind == UPIR_BODY_COVER ? 0
                  : kind == UPIR_BODY_SUM                           ? 1
                  : kind == UPIR_BODY_JACOBI5 || kind == UPIR_BODY_FILTER7 ? 2
                  : kind == UPIR_BODY_MATVEC                        ? 3
                                                                    : 4;
  f[cls] = 1.0f;
  const double n = (double)lp->n;
  double rows = (double)lp->cnt[0], cols = lp->loop.collapse > 1 ? (double)lp->cnt[1] : 1.0, K = 1.0;
  double bpi = 12, fpi = 2;
  if (kind == UPIR_BODY_SUM) bpi = 4, fpi = 1;
  if (kind == UPIR_BODY_COVER) bpi = 8, fpi = 0;
  if (kind == UPIR_BODY_JACOBI5) bpi = 8, fpi = 7;
  if (kind == UPIR_BODY_FILTER7) bpi = 8, fpi = 98;
  if (kind == UPIR_BODY_MATVEC) {
    cols = (double)((const upir_matvec_args *)lp->args)->cols;
    bpi = 4 * cols + 4, fpi = 2 * cols;
  }
  if (is_mm(kind)) {
    K = (double)((const upir_matmul_args *)lp->args)->K;
    bpi = 8.0 * K / 64.0, fpi = 2 * K;
  }
  f[5] = (float)(lg(n) / 32);
  f[6] = (float)(lg(rows) / 32);
  f[7] = (float)(lg(cols) / 32);
  f[8] = (float)(lg(K) / 32);
  f[9] = (float)(lg(bpi) / 32);
  f[10] = (float)(lg(fpi + 1) / 32);
  f[11] = lp->loop.dim[0].step == 1 ? 1.0f : 0.0f;
  f[12] = (float)lp->loop.collapse / 3.0f;
  f[13] = lp->has_red ? 1.0f : 0.0f;
  f[14] = lp->has_red && lp->red.op == UPIR_RED_SUM ? 1.0f : 0.0f;
  f[15] = lp->has_red && lp->red.op != UPIR_RED_SUM ? 1.0f : 0.0f;
  // candidate
  const double U = k.sp.num_units > 0 ? k.sp.num_units : 256;
  f[16] = (float)(lg(U) / 10);
  f[17] = (float)(lg(k.sc.tile[0] > 0 ? k.sc.tile[0] : 1) / 10);
  f[18] = (float)(lg(k.sc.tile[1] > 0 ? k.sc.tile[1] : 1) / 10);
  f[19] = (float)(lg(k.sc.chunk > 0 ? (double)k.sc.chunk : 1) / 10);
  double T = k.sp.num_teams;
  if (T <= 0 && k.sc.tile[0] > 0) {
    T = ceil(rows / k.sc.tile[0]) * (lp->loop.collapse > 1 ? ceil(cols / std::max(1, k.sc.tile[1])) : 1.0);
  }
  f[20] = (float)(lg(T) / 24);
  const double items = n / std::max(1.0, T);
  f[21] = (float)(lg(items) / 32);
  f[22] = (float)(lg(items / U) / 16);
  f[23] = (float)std::min(1.0, T / 2048.0);  // occupancy estimate: teams vs resident slots
  f[24] = k.sp.num_teams > 0 ? 0.0f : 1.0f;  // one team per tile
  f[25] = (float)(lg((double)(k.sc.tile[0] > 0 ? k.sc.tile[0] : 1) * (k.sc.tile[1] > 0 ? k.sc.tile[1] : 1)) / 24);
  const double ws = n * bpi;
  f[26] = (float)(lg(ws / 256e6 + 1e-9) / 32);
  // Jacobi: rows of a wavefront's strip (tile rows / wavefronts per team)
  f[27] = ((kind == UPIR_BODY_JACOBI5 || kind == UPIR_BODY_FILTER7) && k.sc.tile[0] > 0) ? (float)(k.sc.tile[0] / std::max(1.0, U / 64) / 64.0) : 0.0f;
  f[28] = (float)(lg(n * bpi) / 40);
  f[29] = (float)(lg(n * fpi + 1) / 48);
  f[30] = 0.0f;
  f[31] = 0.0f;
}

void candidate_features(upir_ctx *, const upir_loop_obj *lp, const upir_spmd &sp, const upir_sched &sc, float f[32]) {
  Cand k{sp, sc};
  features(lp, k, f);
}

// Cost model pick: batch every candidate through one forward pass and take
// the smallest predicted time. Returns false when the model is off.
bool model_pick(upir_ctx *c, upir_loop_obj *lp, upir_spmd &sp, upir_sched &sc) {
  if (!c->model || !c->model_on || c->capturing || c->no_alloc) return false;  // inference allocates
  auto cs = candidates(c, lp);
  if (cs.empty()) return false;
  std::vector<float> X(cs.size() * 32);
  for (size_t i = 0; i < cs.size(); ++i) features(lp, cs[i], &X[i * 32]);
  float *dX = (float *)upir_dalloc(c, X.size() * 4), *dY = (float *)upir_dalloc(c, cs.size() * 4);
  std::vector<float> y(cs.size());
  bool ok = dX && dY;
  if (ok) ok = hipMemcpyAsync(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess;
  if (ok) ok = fwd_launch(c, dX, (int64_t)cs.size(), dY, nullptr, nullptr) == hipSuccess;
  if (ok) ok = hipMemcpyAsync(y.data(), dY, y.size() * 4, hipMemcpyDeviceToHost, c->stream) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(c->stream) == hipSuccess;
  upir_dfree(c, dX);
  upir_dfree(c, dY);
  if (!ok) return false;
  size_t b = 0;
  for (size_t i = 1; i < y.size(); ++i)
    if (y[i] < y[b]) b = i;
  sp = cs[b].sp;
  sc = cs[b].sc;
  return true;
}

// ------------------------------------------------ engine schedules (batched)
std::vector<upir_engine_sched> engine_candidates() {
  std::vector<upir_engine_sched> v;
  v.push_back(upir_engine_sched{16384, 16384, 64});  // the default first
  for (int64_t a : {8192, 16384, 32768})
    for (int64_t s : {16384, 32768, 65536})
      for (int64_t m : {32, 64, 128})
        if (!(a == 16384 && s == 16384 && m == 64)) v.push_back(upir_engine_sched{a, s, m});
  return v;
}

namespace {
// engine class of a task: 0 AXPY / COVER, 1 SUM, 2 MATVEC
int engine_class(int32_t kind) { return kind == UPIR_BODY_SUM ? 1 : (kind == UPIR_BODY_MATVEC ? 2 : 0); }

int64_t task_len(const TaskRec &t) { return t.hi >= 0 ? t.hi - t.lo : t.loop->n; }

double task_bytes(const TaskRec &t) {
  const double n = (double)task_len(t);
  switch (t.loop->kind) {
    case UPIR_BODY_AXPY: return 12.0 * n;
    case UPIR_BODY_SUM: return 4.0 * n;
    case UPIR_BODY_MATVEC: return (4.0 * (double)((const upir_matvec_args *)t.loop->args)->cols + 4.0) * n;
    default: return 8.0 * n;
  }
}

// tile a candidate gives a task of class k (engine work items count rows for MATVEC)
int64_t class_tile(const upir_engine_sched &es, int k) {
  return k == 0 ? es.tile_axpy : (k == 1 ? es.tile_sum : es.rows_matvec);
}
}  // namespace

uint64_t batch_key(const upir_ctx *c) {
  // FNV-1a over the task count, each task's body and length, the edge count
  uint64_t h = 1469598103934665603ULL;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xff;
      h *= 1099511628211ULL;
    }
  };
  mix(0xBA7C4ULL);
  mix((uint64_t)c->tasks.size());
  uint64_t edges = 0;
  for (const TaskRec &t : c->tasks) {
    mix((uint64_t)(t.loop ? t.loop->kind : 0));
    mix((uint64_t)(t.loop ? task_len(t) : 0));
    edges += t.preds.size();
  }
  mix(edges);
  return h;
}

// 32 features of (pending task graph, engine candidate). Slot 30 marks a
// graph row (loop rows leave it 0). The candidate enters as one one-hot per
// body over that body's three tile choices, weighted by the body's share of
// the graph's bytes, so that a choice's effect on the graph's relative cost
// is close to additive in the features; then the work items each body makes.
static const int64_t kEngineOpts[3][3] = {{8192, 16384, 32768}, {16384, 32768, 65536}, {32, 64, 128}};
static int choice_index(int k, int64_t tile) {
  for (int q = 0; q < 3; ++q)
    if (kEngineOpts[k][q] == tile) return q;
  return -1;
}
static int64_t choice_tile(int k, int q) { return kEngineOpts[k][q]; }

void batch_features(const upir_ctx *c, const upir_engine_sched &es, float f[32]) {
  for (int i = 0; i < 32; ++i) f[i] = 0.0f;
  const size_t n = c->tasks.size();
  double cnt[3] = {0, 0, 0}, bytes[3] = {0, 0, 0}, items[3] = {0, 0, 0}, lgsum = 0, lgmax = 0, edges = 0;
  std::vector<int32_t> depth(n, 0);
  int32_t dmax = 0;
  for (size_t j = 0; j < n; ++j) {
    const TaskRec &t = c->tasks[j];
    if (!t.loop) continue;
    const int k = engine_class(t.loop->kind);
    const int64_t len = std::max<int64_t>(task_len(t), 1);
    cnt[k] += 1;
    bytes[k] += task_bytes(t);
    const int64_t tile = std::max<int64_t>(1, class_tile(es, k));
    items[k] += (double)((len + tile - 1) / tile);
    lgsum += lg((double)len);
    lgmax = std::max(lgmax, lg((double)len));
    edges += (double)t.preds.size();
    int32_t d = 0;
    for (int64_t p : t.preds) d = std::max(d, depth[(size_t)p]);
    depth[j] = d + 1;
    dmax = std::max(dmax, depth[j]);
  }
  const double N = std::max<double>(1.0, (double)n), B = std::max(1.0, bytes[0] + bytes[1] + bytes[2]);
  const double I = std::max(1.0, items[0] + items[1] + items[2]), grid = 4.0 * c->num_cus;
  for (int k = 0; k < 3; ++k) {
    f[k] = (float)(cnt[k] / N);
    f[3 + k] = (float)(bytes[k] / B);
    const int q = choice_index(k, class_tile(es, k));
    if (q >= 0) f[12 + 3 * k + q] = (float)(bytes[k] / B);
    f[21 + k] = (float)(lg(items[k] + 1) / 24);
  }
  f[6] = (float)(lg(N) / 16);
  f[7] = (float)(lg(B) / 40);
  f[8] = (float)(lgsum / N / 32);
  f[9] = (float)(lgmax / 32);
  f[10] = (float)(edges / N / 8);
  f[11] = (float)(dmax / 64.0);
  f[24] = (float)(lg(I / grid) / 16);
  f[30] = 1.0f;
}

// Cost model pick of the engine schedule for the pending task graph: one
// forward pass over the 27 candidates, then the choice below. Returns false
// when the model is off.
bool model_pick_engine(upir_ctx *c, upir_engine_sched &es) {
  if (!c->model || !c->model_on || c->capturing || c->no_alloc || c->tasks.empty()) return false;
  const auto cs = engine_candidates();
  std::vector<float> X(cs.size() * 32), y(cs.size());
  for (size_t i = 0; i < cs.size(); ++i) batch_features(c, cs[i], &X[i * 32]);
  float *dX = (float *)upir_dalloc(c, X.size() * 4), *dY = (float *)upir_dalloc(c, cs.size() * 4);
  bool ok = dX && dY;
  if (ok) ok = hipMemcpyAsync(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice, c->stream) == hipSuccess;
  if (ok) ok = fwd_launch(c, dX, (int64_t)cs.size(), dY, nullptr, nullptr) == hipSuccess;
  if (ok) ok = hipMemcpyAsync(y.data(), dY, y.size() * 4, hipMemcpyDeviceToHost, c->stream) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(c->stream) == hipSuccess;
  upir_dfree(c, dX);
  upir_dfree(c, dY);
  if (!ok) return false;
  // The choice is among the schedules the exhaustive batch tuner found best
  // on the (up to) ten tuned graphs most like this one, and the default.
  // Graphs are compared by their candidate-independent features (task and
  // byte shares per body, task count, bytes, lengths, edges, depth). Each
  // such schedule is scored by the model's prediction plus the mean of its
  // measured log2(time / default) over those graphs (the tuner timed every
  // candidate on them). On its own the model's error is of the order of the
  // differences it has to rank (the candidates of a large graph lie within
  // a few percent of each other): its argmin over all 27 sometimes took a
  // schedule that tuned graphs of another kind preferred (smaller graphs
  // favour smaller matvec tiles), and ranking only the nearest graphs' best
  // schedules by the prediction still flipped between two of them from one
  // trained model to the next. Without tuned graphs, each body takes the
  // tile whose candidates have the lowest mean prediction over the other
  // bodies' choices (nine predictions per mean).
  auto same = [](const upir_engine_sched &a, const upir_engine_sched &b) {
    return a.tile_axpy == b.tile_axpy && a.tile_sum == b.tile_sum && a.rows_matvec == b.rows_matvec;
  };
  struct Near {
    float d;
    upir_engine_sched best;
    const std::vector<float> *rel;
  };
  std::vector<Near> near;
  for (const auto &kv : c->tuned_engine) {
    auto g = c->tuned_engine_graph.find(kv.first);
    if (g == c->tuned_engine_graph.end()) continue;
    auto r = c->tuned_engine_rel.find(kv.first);
    float d = 0.0f;
    for (int q = 0; q < 12; ++q) d += (g->second[(size_t)q] - X[(size_t)q]) * (g->second[(size_t)q] - X[(size_t)q]);
    near.push_back(Near{d, kv.second.first,
                        r != c->tuned_engine_rel.end() && r->second.size() == cs.size() ? &r->second : nullptr});
  }
  const size_t kn = std::min<size_t>(10, near.size());
  std::partial_sort(near.begin(), near.begin() + (ptrdiff_t)kn, near.end(),
                    [](const Near &a, const Near &b) { return a.d < b.d; });
  int pick = -1, seen = 0;
  float pick_score = 0.0f;
  for (size_t i = 0; i < cs.size(); ++i) {
    bool in = i == 0;  // candidate 0, the default, always takes part
    for (size_t j = 0; j < kn && !in; ++j) in = same(near[j].best, cs[i]);
    if (!in) continue;
    seen += i > 0;
    double m = 0.0;
    int nm = 0;
    for (size_t j = 0; j < kn; ++j)
      if (near[j].rel) {
        m += (*near[j].rel)[i];
        ++nm;
      }
    const float score = y[i] + (nm ? (float)(m / nm) : 0.0f);
    if (pick < 0 || score < pick_score) {
      pick = (int)i;
      pick_score = score;
    }
  }
  if (seen > 0) {
    es = cs[(size_t)pick];
    return true;
  }
  double sum[3][3] = {}, cnt[3][3] = {};
  for (size_t i = 0; i < cs.size(); ++i)
    for (int k = 0; k < 3; ++k) {
      const int q = choice_index(k, class_tile(cs[i], k));
      if (q < 0) continue;
      sum[k][q] += y[i];
      cnt[k][q] += 1;
    }
  int best[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k)
    for (int q = 1; q < 3; ++q)
      if (cnt[k][q] > 0 && (cnt[k][best[k]] == 0 || sum[k][q] / cnt[k][q] < sum[k][best[k]] / cnt[k][best[k]])) best[k] = q;
  es = upir_engine_sched{choice_tile(0, best[0]), choice_tile(1, best[1]), choice_tile(2, best[2])};
  return true;
}

upir_status resolve_engine_sched(upir_ctx *c, upir_engine_sched &es, int32_t &source) {
  if (c->engine_set) {
    es = c->engine_sched;
    source = UPIR_ENGINE_FROM_CALLER;
    return UPIR_OK;
  }
  auto it = c->tuned_engine.find(batch_key(c));
  if (it != c->tuned_engine.end()) {
    es = it->second.first;
    source = UPIR_ENGINE_FROM_TUNER;
    return UPIR_OK;
  }
  if (model_pick_engine(c, es)) {
    source = UPIR_ENGINE_FROM_MODEL;
    return UPIR_OK;
  }
  es = engine_candidates()[0];
  source = UPIR_ENGINE_FROM_DEFAULT;
  return UPIR_OK;
}

}  // namespace upir

extern "C" upir_status upir_engine_sched_set(upir_ctx *c, const upir_engine_sched *es) {
  if (!c) return UPIR_EINVAL;
  if (!es) {
    c->engine_set = false;
    return UPIR_OK;
  }
  for (int64_t t : {es->tile_axpy, es->tile_sum, es->rows_matvec})
    if (t < 1 || t > (1 << 24)) return upir_fail(c, UPIR_EINVAL, "engine tile %lld", (long long)t);
  c->engine_sched = *es;
  c->engine_set = true;
  return UPIR_OK;
}

extern "C" upir_status upir_engine_sched_resolve(upir_ctx *c, upir_engine_sched *out, int32_t *source) {
  if (!c || !out) return UPIR_EINVAL;
  int32_t src = 0;
  upir_status st = resolve_engine_sched(c, *out, src);
  if (source) *source = src;
  return st;
}

extern "C" upir_status upir_engine_candidate(upir_ctx *c, int32_t idx, upir_engine_sched *out, float *feat) {
  if (!c || !out) return UPIR_EINVAL;
  const auto cs = engine_candidates();
  if (idx < 0 || idx >= (int)cs.size()) return upir_fail(c, UPIR_EINVAL, "engine candidate %d of %zu", idx, cs.size());
  *out = cs[idx];
  if (feat) batch_features(c, cs[idx], feat);
  return UPIR_OK;
}

// ------------------------------------------------------------------- tuner
extern "C" upir_status upir_candidates(upir_ctx *c, upir_loop_h lp, int32_t *count) {
  if (!c || !lp || !count || !c->loops.count(lp)) return UPIR_EINVAL;
  *count = candidate_count(c, lp);
  return UPIR_OK;
}

extern "C" upir_status upir_candidate_features(upir_ctx *c, upir_loop_h lp, int32_t idx, float *feat,
                                               upir_spmd *sp_out, upir_sched *sc_out) {
  if (!c || !lp || !c->loops.count(lp)) return UPIR_EINVAL;
  auto cs = candidates(c, lp);
  if (idx < 0 || idx >= (int)cs.size()) return upir_fail(c, UPIR_EINVAL, "candidate %d of %zu", idx, cs.size());
  if (feat) features(lp, cs[idx], feat);
  if (sp_out) *sp_out = cs[idx].sp;
  if (sc_out) *sc_out = cs[idx].sc;
  return UPIR_OK;
}

// Run `lp` under candidate k `reps` times; median time in microseconds.
static upir_status time_candidate(upir_ctx *c, upir_loop_obj *tmp, const Cand &k, int reps, double &us) {
  tmp->sched = k.sc;
  Plan pl;
  upir_status st = resolve_plan(c, &k.sp, tmp, pl);
  if (st) return st;
  if (tmp->has_red) {  // size the reduction slots first; the result slot moves with them
    st = ensure_scratch(c, tmp, pl.S.T);
    if (st) return st;
    tmp->red.result = tmp->scratch + SCR_RESULT;
  }
  st = launch_plan(c, tmp, pl, false);  // warm-up
  if (st) return st;
  std::vector<float> ms;
  hipEvent_t a, b;
  HIPTRY(c, hipEventCreate(&a));
  HIPTRY(c, hipEventCreate(&b));
  for (int r = 0; r < reps && st == UPIR_OK; ++r) {
    if (hipEventRecord(a, c->stream) != hipSuccess) {
      st = upir_fail(c, UPIR_EHIP, "event record");
      break;
    }
    st = launch_plan(c, tmp, pl, false);
    if (st) break;
    float t = 0;
    if (hipEventRecord(b, c->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&t, a, b) != hipSuccess)
      st = upir_fail(c, UPIR_EHIP, "event wait");
    ms.push_back(t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st) return st;
  std::sort(ms.begin(), ms.end());
  us = 1e3 * ms[ms.size() / 2];
  return UPIR_OK;
}

extern "C" upir_status upir_tune(upir_ctx *c, const upir_spmd *spmd, upir_loop_h lp, int32_t reps, upir_sched *best,
                                 upir_spmd *best_spmd, double *best_us) {
  (void)spmd;
  if (!c || !lp || !c->loops.count(lp)) return UPIR_EINVAL;
  if (c->none) return upir_fail(c, UPIR_ESTATE, "host-only context");
  if (c->capturing) return upir_fail(c, UPIR_ESTATE, "tuning during graph capture");
  if (reps < 1 || reps > 1000) return upir_fail(c, UPIR_EINVAL, "reps");
  {
    upir_status s0 = settle(c);
    if (s0) return s0;
  }
  // scratch copies of read-write outputs, and an internal reduction result
  upir_loop_obj tmp = *lp;
  tmp.scratch = nullptr;
  tmp.part_cap = 0;
  tmp.ws = lp->ws;
  unsigned char pay[sizeof(MatmulP) + 16];
  upir_status st = resolve_payload(c, lp, pay);
  if (st) return st;
  tmp.args_dev = 1;
  std::vector<void *> owned;
  auto own = [&](size_t bytes) -> void * {
    void *p = upir_dalloc(c, bytes);
    if (p) owned.push_back(p);
    return p;
  };
  auto cleanup = [&]() {
    (void)settle(c);  // a deferred fold of the copy writes into its scratch
    (void)hipStreamSynchronize(c->stream);
    for (void *p : owned) upir_dfree(c, p);
    upir_dfree(c, tmp.scratch);
  };
  // extent (elements) of the index range a 1-D loop touches
  int64_t lo = lp->loop.dim[0].lb, hi = lo + (lp->n > 0 ? (lp->n - 1) * lp->loop.dim[0].step : 0);
  if (hi < lo) std::swap(lo, hi);
  const size_t span1 = (size_t)(hi + 1);
  switch (lp->kind) {
    case UPIR_BODY_AXPY: {  // y is read and written: time on a copy
      const AxpyP &p = *(const AxpyP *)pay;
      float *y2 = (float *)own(span1 * 4);
      if (!y2) break;
      if (lp->n > 0) (void)hipMemcpyAsync(y2, p.y, span1 * 4, hipMemcpyDeviceToDevice, c->stream);
      upir_axpy_args a{p.a, 0, p.x, y2};
      memcpy(tmp.args, &a, sizeof a);
      break;
    }
    case UPIR_BODY_COVER: {
      int32_t *c2 = (int32_t *)own((size_t)std::max<int64_t>(lp->n, 1) * 4);
      if (!c2) break;
      upir_cover_args a{c2};
      memcpy(tmp.args, &a, sizeof a);
      break;
    }
    case UPIR_BODY_SUM: {
      const SumP &p = *(const SumP *)pay;
      upir_sum_args a{p.x, p.dtype, 0};
      memcpy(tmp.args, &a, sizeof a);
      break;
    }
    case UPIR_BODY_JACOBI5: {  // dst on a scratch grid of the same pitch
      const JacobiP &p = *(const JacobiP *)pay;
      const int64_t rows = lp->loop.dim[0].lb + lp->cnt[0] + 1;
      float *d2 = (float *)own((size_t)rows * p.ld * 4);
      if (!d2) break;
      upir_jacobi5_args a{p.src, d2, p.ld};
      memcpy(tmp.args, &a, sizeof a);
      break;
    }
    case UPIR_BODY_FILTER7: {  // dst on a scratch grid of the same pitch
      const Filter7P &p = *(const Filter7P *)pay;
      const int64_t rows = lp->loop.dim[0].lb + lp->cnt[0] + 3;
      float *d2 = (float *)own((size_t)rows * p.ld * 4);
      if (!d2) break;
      upir_filter7_args a{p.src, d2, p.w, p.ld};
      memcpy(tmp.args, &a, sizeof a);
      break;
    }
    case UPIR_BODY_MATVEC: {
      const MatvecP &p = *(const MatvecP *)pay;
      float *y2 = (float *)own(span1 * 4);
      if (!y2) break;
      upir_matvec_args a{p.A, p.x, y2, p.cols, p.lda};
      memcpy(tmp.args, &a, sizeof a);
      break;
    }
    case UPIR_BODY_OWNER: {
      int32_t *o2 = (int32_t *)own((size_t)std::max<int64_t>(lp->n, 1) * 4);
      if (!o2) break;
      upir_owner_args a{o2};
      memcpy(tmp.args, &a, sizeof a);
      break;
    }
    default: {  // matmul: C on a scratch matrix, BF16 workspace of the loop
      const MatmulP &p = *(const MatmulP *)pay;
      float *c2 = (float *)own((size_t)std::max<int64_t>(p.M, 1) * p.ldc * 4);
      if (!c2) break;
      upir_matmul_args a = *(const upir_matmul_args *)lp->args;
      a.A = p.A;
      a.B = p.B;
      a.C = c2;
      a.workspace = p.ah;
      a.workspace_bytes = upir_matmul_workspace_bytes(lp->kind, p.M, p.N, p.K);
      memcpy(tmp.args, &a, sizeof a);
    }
  }
  if (owned.empty() && lp->kind != UPIR_BODY_SUM) {
    cleanup();
    return upir_fail(c, UPIR_ENOMEM, "tuner scratch");
  }
  if (lp->has_red) {
    tmp.red.result_on_host = 0;
    tmp.part_cap = 0;
  }
  tmp.part_cap = tmp.has_red ? 8192 : 0;
  tmp.scratch = (unsigned char *)upir_dalloc(c, scratch_bytes(tmp.part_cap));
  if (!tmp.scratch) {
    cleanup();
    return upir_fail(c, UPIR_ENOMEM, "tuner scratch");
  }
  st = clear_scratch(c, &tmp, tmp.scratch, tmp.part_cap);
  if (st) {
    cleanup();
    return st;
  }
  if (tmp.has_red) tmp.red.result = tmp.scratch + SCR_RESULT;
  auto cs = candidates(c, lp);
  double bus = 1e300;
  int bi = -1;
  for (int i = 0; i < (int)cs.size(); ++i) {
    double us = 0;
    st = time_candidate(c, &tmp, cs[i], reps, us);
    if (st) break;
    TuneRow row{};
    features(lp, cs[i], row.feat);
    row.log2_us = (float)log2(std::max(us, 1e-3));
    row.loop_key = (int64_t)(lp->key & 0x7FFFFFFFFFFFFFFFULL);
    c->db.push_back(row);
    if (us < bus) {
      bus = us;
      bi = i;
    }
  }
  cleanup();
  if (st) return st;
  if (bi < 0) return upir_fail(c, UPIR_EUNSUPPORTED, "no candidate schedules for this loop");
  c->tuned[lp->key] = TunedChoice{cs[bi].sp, cs[bi].sc, bus};
  if (best) *best = cs[bi].sc;
  if (best_spmd) *best_spmd = cs[bi].sp;
  if (best_us) *best_us = bus;
  return UPIR_OK;
}
