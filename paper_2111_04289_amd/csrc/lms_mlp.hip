// Learned placement cost model: a 12 -> 64 -> 64 -> 2 ReLU MLP that predicts
// log(CPU ms) and log(GPU ms) of an operation from its features.  It replaces
// the analytic device costs of Eq. 7-9 (and the InfPT regression of Eq. 10) in
// MapDevice (Algorithm 2) when lms_plan runs in LMS_PLAN_LEARNED mode.
//
// Training runs on the GPU with hand-written kernels: a fused forward/backward
// pass per tile of 64 samples (weights, activations and their gradients held
// in LDS), a deterministic reduction of the per-tile gradients, and an Adam
// step.  Inference runs on the GPU in FP32 or with BF16 weights, and on the
// host (for the synchronous lms_plan) in FP32.
#include <cmath>
#include <cstring>
#include <vector>

#include "lms_internal.h"

namespace lms {
namespace {

constexpr int IN = LMS_MLP_IN, HID = LMS_MLP_HIDDEN, OUT = LMS_MLP_OUT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + HID * IN, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + OUT * HID, NP = OFF_B3 + OUT;
static_assert(NP == LMS_MLP_NPARAMS, "parameter layout");
constexpr int TILE = 64;  // samples per workgroup
constexpr int TPB = 256;

// Round-to-nearest-even FP32 -> BF16 -> FP32 (NaN kept as NaN).
__host__ __device__ inline float bf16_round(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return f;
  u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  float r;
  memcpy(&r, &u, 4);
  return r;
}

// Fused forward + backward of the masked squared error
//   L = (1/n) sum_s sum_o mask[s,o] * (y[s,o] - t[s,o])^2
// for one tile of samples; writes this tile's gradient and loss partials.
__global__ __launch_bounds__(TPB) void k_mlp_fwd_bwd(const float* __restrict__ params, const float* __restrict__ x,
                                                      const float* __restrict__ t, const float* __restrict__ mask,
                                                      int64_t n, float* __restrict__ gpart, float* __restrict__ lpart) {
  __shared__ float w[NP];
  __shared__ float xs[TILE][IN];
  __shared__ float h1[TILE][HID];
  __shared__ float h2[TILE][HID];  // later reused for dh1
  __shared__ float dh[TILE][HID];  // dh2
  __shared__ float dy[TILE][OUT];
  __shared__ float lsum[TPB];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * TILE;
  for (int i = tid; i < NP; i += TPB) w[i] = params[i];
  for (int i = tid; i < TILE * IN; i += TPB) {
    const int s = i / IN, k = i % IN;
    xs[s][k] = s0 + s < n ? x[(s0 + s) * IN + k] : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < TILE * HID; i += TPB) {  // h1 = relu(W1 x + b1)
    const int s = i / HID, j = i % HID;
    float a = w[OFF_B1 + j];
    for (int k = 0; k < IN; ++k) a += w[OFF_W1 + j * IN + k] * xs[s][k];
    h1[s][j] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < TILE * HID; i += TPB) {  // h2 = relu(W2 h1 + b2)
    const int s = i / HID, j = i % HID;
    float a = w[OFF_B2 + j];
    for (int k = 0; k < HID; ++k) a += w[OFF_W2 + j * HID + k] * h1[s][k];
    h2[s][j] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  float lacc = 0.f;
  const float inv_n = 1.f / (float)n;
  for (int i = tid; i < TILE * OUT; i += TPB) {  // y = W3 h2 + b3; dL/dy
    const int s = i / OUT, o = i % OUT;
    float y = w[OFF_B3 + o];
    for (int k = 0; k < HID; ++k) y += w[OFF_W3 + o * HID + k] * h2[s][k];
    float g = 0.f;
    if (s0 + s < n) {
      const float m = mask[(s0 + s) * OUT + o];
      const float d = y - t[(s0 + s) * OUT + o];
      lacc += m * d * d * inv_n;
      g = 2.f * m * d * inv_n;
    }
    dy[s][o] = g;
  }
  lsum[tid] = lacc;
  __syncthreads();
  float* gp = gpart + (size_t)blockIdx.x * NP;
  for (int i = tid; i < OUT * HID + OUT; i += TPB) {  // dW3, db3
    if (i < OUT * HID) {
      const int o = i / HID, j = i % HID;
      float a = 0.f;
      for (int s = 0; s < TILE; ++s) a += dy[s][o] * h2[s][j];
      gp[OFF_W3 + i] = a;
    } else {
      const int o = i - OUT * HID;
      float a = 0.f;
      for (int s = 0; s < TILE; ++s) a += dy[s][o];
      gp[OFF_B3 + o] = a;
    }
  }
  for (int i = tid; i < TILE * HID; i += TPB) {  // dh2 = (W3^T dy) * relu'(h2)
    const int s = i / HID, j = i % HID;
    float a = 0.f;
    for (int o = 0; o < OUT; ++o) a += w[OFF_W3 + o * HID + j] * dy[s][o];
    dh[s][j] = h2[s][j] > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < HID * HID + HID; i += TPB) {  // dW2, db2
    if (i < HID * HID) {
      const int r = i / HID, c = i % HID;
      float a = 0.f;
      for (int s = 0; s < TILE; ++s) a += dh[s][r] * h1[s][c];
      gp[OFF_W2 + i] = a;
    } else {
      const int r = i - HID * HID;
      float a = 0.f;
      for (int s = 0; s < TILE; ++s) a += dh[s][r];
      gp[OFF_B2 + r] = a;
    }
  }
  for (int i = tid; i < TILE * HID; i += TPB) {  // dh1 = (W2^T dh2) * relu'(h1), stored in h2
    const int s = i / HID, j = i % HID;
    float a = 0.f;
    for (int r = 0; r < HID; ++r) a += w[OFF_W2 + r * HID + j] * dh[s][r];
    h2[s][j] = h1[s][j] > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < HID * IN + HID; i += TPB) {  // dW1, db1
    if (i < HID * IN) {
      const int j = i / IN, k = i % IN;
      float a = 0.f;
      for (int s = 0; s < TILE; ++s) a += h2[s][j] * xs[s][k];
      gp[OFF_W1 + i] = a;
    } else {
      const int j = i - HID * IN;
      float a = 0.f;
      for (int s = 0; s < TILE; ++s) a += h2[s][j];
      gp[OFF_B1 + j] = a;
    }
  }
  if (tid == 0) {
    float l = 0.f;
    for (int k = 0; k < TPB; ++k) l += lsum[k];
    lpart[blockIdx.x] = l;
  }
}

// grad[p] = sum over tiles of the partials, in tile order (deterministic).
__global__ void k_mlp_reduce(const float* __restrict__ gpart, const float* __restrict__ lpart, int ntiles,
                             float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) {
    float a = 0.f;
    for (int tt = 0; tt < ntiles; ++tt) a += gpart[(size_t)tt * NP + p];
    grad[p] = a;
  }
  if (p == 0 && loss) {
    float l = 0.f;
    for (int tt = 0; tt < ntiles; ++tt) l += lpart[tt];
    *loss = l;
  }
}

__global__ void k_mlp_adam(float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ grad, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Inference: one thread per sample, weights (FP32 or BF16-rounded) and the
// first hidden layer in LDS (laid out [unit][thread], conflict-free).
__global__ __launch_bounds__(TPB) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ x,
                                                      int64_t n, float* __restrict__ y, int use_bf16) {
  __shared__ float w[NP];
  __shared__ float act[HID][TPB];
  for (int i = threadIdx.x; i < NP; i += TPB) w[i] = use_bf16 ? bf16_round(params[i]) : params[i];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (s >= n) return;
  float xi[IN];
#pragma unroll
  for (int k = 0; k < IN; ++k) xi[k] = x[s * IN + k];
  for (int j = 0; j < HID; ++j) {
    float a = w[OFF_B1 + j];
#pragma unroll
    for (int k = 0; k < IN; ++k) a += w[OFF_W1 + j * IN + k] * xi[k];
    act[j][threadIdx.x] = a > 0.f ? a : 0.f;
  }
  float o0 = w[OFF_B3], o1 = w[OFF_B3 + 1];
  for (int j = 0; j < HID; ++j) {
    float a = w[OFF_B2 + j];
    for (int k = 0; k < HID; ++k) a += w[OFF_W2 + j * HID + k] * act[k][threadIdx.x];
    a = a > 0.f ? a : 0.f;
    o0 += w[OFF_W3 + j] * a;
    o1 += w[OFF_W3 + HID + j] * a;
  }
  y[s * OUT] = o0;
  y[s * OUT + 1] = o1;
}

}  // namespace

// Host forward pass of the same network (used by the synchronous planner).
void mlp_host_forward(const float* p, const float* x, float* y) {
  float a1[HID];
  for (int j = 0; j < HID; ++j) {
    float a = p[OFF_B1 + j];
    for (int k = 0; k < IN; ++k) a += p[OFF_W1 + j * IN + k] * x[k];
    a1[j] = a > 0.f ? a : 0.f;
  }
  float o0 = p[OFF_B3], o1 = p[OFF_B3 + 1];
  for (int j = 0; j < HID; ++j) {
    float a = p[OFF_B2 + j];
    for (int k = 0; k < HID; ++k) a += p[OFF_W2 + j * HID + k] * a1[k];
    a = a > 0.f ? a : 0.f;
    o0 += p[OFF_W3 + j] * a;
    o1 += p[OFF_W3 + HID + j] * a;
  }
  y[0] = o0;
  y[1] = o1;
}

}  // namespace lms

using namespace lms;

struct lms_mlp {
  float* params;  // device, NP
  float* m;       // Adam first moment
  float* v;       // Adam second moment
  int64_t step;
};

extern "C" int lms_mlp_create(uint64_t seed, lms_mlp** out) {
  if (!out) return set_error(LMS_EINVAL, "out is NULL");
  *out = nullptr;
  // He-uniform initialisation from a counter-based generator (SplitMix64 of
  // seed and parameter index); biases start at zero.
  std::vector<float> h(NP, 0.f);
  auto uni = [&](uint64_t i) {
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + i + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  };
  auto fill = [&](int off, int fan_out, int fan_in) {
    const double lim = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < fan_out * fan_in; ++i) h[off + i] = (float)(lim * uni((uint64_t)(off + i)));
  };
  fill(OFF_W1, HID, IN);
  fill(OFF_W2, HID, HID);
  fill(OFF_W3, OUT, HID);
  lms_mlp* m = new lms_mlp{};
  int rc = check_hip(hipMalloc(&m->params, NP * sizeof(float)), "hipMalloc mlp");
  if (!rc) rc = check_hip(hipMalloc(&m->m, NP * sizeof(float)), "hipMalloc mlp");
  if (!rc) rc = check_hip(hipMalloc(&m->v, NP * sizeof(float)), "hipMalloc mlp");
  if (!rc) rc = check_hip(hipMemcpy(m->params, h.data(), NP * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  if (!rc) rc = check_hip(hipMemset(m->m, 0, NP * sizeof(float)), "hipMemset");
  if (!rc) rc = check_hip(hipMemset(m->v, 0, NP * sizeof(float)), "hipMemset");
  if (rc) {
    lms_mlp_free(m);
    return rc;
  }
  *out = m;
  return LMS_OK;
}

extern "C" void lms_mlp_free(lms_mlp* m) {
  if (!m) return;
  hipFree(m->params);
  hipFree(m->m);
  hipFree(m->v);
  delete m;
}

extern "C" int lms_mlp_set_params(lms_mlp* m, const float* host_params) {
  if (!m || !host_params) return set_error(LMS_EINVAL, "NULL argument");
  m->step = 0;
  int rc = check_hip(hipMemcpy(m->params, host_params, NP * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  if (!rc) rc = check_hip(hipMemset(m->m, 0, NP * sizeof(float)), "hipMemset");
  if (!rc) rc = check_hip(hipMemset(m->v, 0, NP * sizeof(float)), "hipMemset");
  return rc;
}

extern "C" int lms_mlp_get_params(const lms_mlp* m, float* host_params) {
  if (!m || !host_params) return set_error(LMS_EINVAL, "NULL argument");
  return check_hip(hipMemcpy(host_params, m->params, NP * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
}

extern "C" size_t lms_mlp_workspace(int64_t n) {
  const int64_t tiles = (n + TILE - 1) / TILE;
  return align_up((size_t)std::max<int64_t>(1, tiles) * NP * sizeof(float), 256) +
         align_up((size_t)std::max<int64_t>(1, tiles) * sizeof(float), 256);
}

extern "C" int lms_mlp_loss_grad(const lms_mlp* m, const float* d_x, const float* d_t, const float* d_mask, int64_t n,
                                 float* d_grad, float* d_loss, void* workspace, size_t ws_bytes, lms_stream stream) {
  if (!m || !d_x || !d_t || !d_mask || !d_grad || n <= 0) return set_error(LMS_EINVAL, "bad MLP training arguments");
  if (n >= (int64_t(1) << 31)) return set_error(LMS_EINVAL, "too many samples");
  if (!workspace || ws_bytes < lms_mlp_workspace(n)) return set_error(LMS_ENOMEM, "workspace too small");
  const int tiles = (int)((n + TILE - 1) / TILE);
  float* gpart = (float*)workspace;
  float* lpart = (float*)((char*)workspace + align_up((size_t)tiles * NP * sizeof(float), 256));
  hipStream_t st = (hipStream_t)stream;
  LMS_LAUNCH("k_mlp_fwd_bwd", k_mlp_fwd_bwd, dim3(tiles), dim3(TPB), 0, st, m->params, d_x, d_t, d_mask, n, gpart,
             lpart);
  LMS_LAUNCH("k_mlp_reduce", k_mlp_reduce, dim3((NP + 255) / 256), dim3(256), 0, st, gpart, lpart, tiles, d_grad,
             d_loss);
  return check_hip(hipGetLastError(), "mlp loss_grad launch");
}

extern "C" int lms_mlp_adam_step(lms_mlp* m, const float* d_grad, float lr, float beta1, float beta2, float eps,
                                 lms_stream stream) {
  if (!m || !d_grad) return set_error(LMS_EINVAL, "NULL argument");
  m->step += 1;
  const float c1 = 1.f - std::pow(beta1, (float)m->step);
  const float c2 = 1.f - std::pow(beta2, (float)m->step);
  LMS_LAUNCH("k_mlp_adam", k_mlp_adam, dim3((NP + 255) / 256), dim3(256), 0, (hipStream_t)stream, m->params, m->m,
             m->v, d_grad, lr, beta1, beta2, eps, c1, c2);
  return check_hip(hipGetLastError(), "mlp adam launch");
}

extern "C" int lms_mlp_forward(const lms_mlp* m, const float* d_x, int64_t n, float* d_y, int32_t use_bf16,
                               lms_stream stream) {
  if (!m || (n > 0 && (!d_x || !d_y)) || n < 0) return set_error(LMS_EINVAL, "bad MLP inference arguments");
  if (n == 0) return LMS_OK;
  LMS_LAUNCH("k_mlp_forward", k_mlp_forward, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0,
             (hipStream_t)stream, m->params, d_x, n, d_y, use_bf16 ? 1 : 0);
  return check_hip(hipGetLastError(), "mlp forward launch");
}

extern "C" void lms_mlp_host_forward(const float* host_params, const float* x, float* y) {
  mlp_host_forward(host_params, x, y);
}

extern "C" float lms_bf16_round(float f) { return bf16_round(f); }

extern "C" void lms_mlp_features(const lms_op_desc* op, const lms_batch_stats* st, int32_t transfer, float* x) {
  for (int k = 0; k < IN; ++k) x[k] = 0.f;
  x[0] = (float)(std::log2((double)st->rows + 1.0) / 24.0);
  x[1] = (float)op->ncols / 8.f;
  x[2] = (float)st->selectivity;
  x[3] = (float)(std::log2((double)st->distinct_keys + 1.0) / 20.0);
  int cls = 0;
  if (op->kind == LMS_OP_JOIN) cls = 3;
  else if (op->kind == LMS_OP_AGG || op->kind == LMS_OP_EXPAND)
    cls = (op->slide_s > 0 && op->slide_s < op->window_s) ? 2 : 1;
  x[4 + cls] = 1.f;
  x[8] = (float)(op->window_s / 60.0);
  x[9] = (float)(op->slide_s / 60.0);
  x[10] = (float)(st->interval_s / 10.0);
  x[11] = transfer ? 1.f : 0.f;
}

namespace lms {
// MapDevice with learned costs: Algorithm 2's walk over the chain, where the
// transfer condition (first or last operation, or the previous one on the CPU)
// is a model input and each operation takes the device predicted faster.
int plan_learned(const lms_op_desc* ops, int32_t nops, const lms_batch_stats* st, const lms_cost_params* cp,
                 int32_t* out_dev, double* out_cost) {
  const lms_mlp_model* model = (const lms_mlp_model*)cp->model;
  for (int o = 0; o < nops; ++o) {
    const int transfer = (o == 0 || o == nops - 1 || out_dev[o - 1] == LMS_DEV_CPU) ? 1 : 0;
    float x[IN], y[OUT];
    lms_mlp_features(&ops[o], st, transfer, x);
    mlp_host_forward(model->params, x, y);
    out_dev[o] = y[1] > y[0] ? LMS_DEV_CPU : LMS_DEV_GPU;
    if (out_cost) out_cost[o] = std::exp((double)(out_dev[o] == LMS_DEV_CPU ? y[0] : y[1]));
  }
  return LMS_OK;
}
}  // namespace lms
