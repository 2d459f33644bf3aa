// Learned direction switch: training-sample collection, the MLP training
// kernel (forward, backward, Adam, loss), test hooks and weight loading.
//
// Training runs in one workgroup: a batch is processed in sub-batches of 64
// samples (one thread per sample for the forward and backward passes, the
// activations staged in LDS), and every gradient entry is summed over the
// samples in a fixed order by the thread that owns that parameter, so
// training is bit-reproducible run to run.  Loss: mean over the batch of
// half the squared error of the two outputs; Adam with bias correction.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/rbfs.h"
#include "common.h"
#include "graph.h"
#include "mlp_dev.h"
#include "switch.h"

namespace rbfs {

static float* s_switch_dev = nullptr;
static int s_switch_device = -1;

const float* switch_blob_device(int device) {
  return (s_switch_dev && s_switch_device == device) ? s_switch_dev : nullptr;
}

namespace {

constexpr int kTrainThreads = 256;
constexpr int kForwardThreads = 256;  // rbfs_mlp_forward: one wave per sample
constexpr int kSub = 64;  // samples per sub-batch
constexpr int kSampleW = kMlpIn + kMlpOut;
constexpr int kParamsPerThread = (kMlpParams + kTrainThreads - 1) / kTrainThreads;

struct TrainLds {
  float w[kMlpParams];
  float x[kSub][kMlpIn];
  float h1[kSub][kMlpHid];
  float h2[kSub][kMlpHid];
  float d1[kSub][kMlpHid];
  float d2[kSub][kMlpHid];
  float dy[kSub][kMlpOut];
  float loss[kSub];
};

// Forward + backward of sample row s (thread s < cnt) of a sub-batch;
// dy is scaled by 1/B for a batch of B samples.
__device__ void sample_pass(TrainLds& L, const float* sample, int s, float invB) {
  float x[kMlpIn];
  for (int k = 0; k < kMlpIn; ++k) {
    x[k] = sample[k];
    L.x[s][k] = x[k];
  }
  float h1[kMlpHid], h2[kMlpHid];
  for (int j = 0; j < kMlpHid; ++j) {
    float a = L.w[kOffB1 + j];
    for (int k = 0; k < kMlpIn; ++k) a = fmaf(L.w[kOffW1 + j * kMlpIn + k], x[k], a);
    h1[j] = fmaxf(a, 0.0f);
    L.h1[s][j] = h1[j];
  }
  for (int j = 0; j < kMlpHid; ++j) {
    float c = L.w[kOffB2 + j];
    for (int k = 0; k < kMlpHid; ++k) c = fmaf(L.w[kOffW2 + j * kMlpHid + k], h1[k], c);
    h2[j] = fmaxf(c, 0.0f);
    L.h2[s][j] = h2[j];
  }
  float y[kMlpOut], dy[kMlpOut];
  float loss = 0.0f;
  for (int o = 0; o < kMlpOut; ++o) {
    float t = L.w[kOffB3 + o];
    for (int k = 0; k < kMlpHid; ++k) t = fmaf(L.w[kOffW3 + o * kMlpHid + k], h2[k], t);
    y[o] = t;
    const float err = t - sample[kMlpIn + o];
    loss = fmaf(0.5f * err, err, loss);
    dy[o] = err * invB;
    L.dy[s][o] = dy[o];
  }
  L.loss[s] = loss;
  for (int j = 0; j < kMlpHid; ++j) {
    float g = 0.0f;
    for (int o = 0; o < kMlpOut; ++o) g = fmaf(L.w[kOffW3 + o * kMlpHid + j], dy[o], g);
    L.d2[s][j] = h2[j] > 0.0f ? g : 0.0f;
  }
  for (int k = 0; k < kMlpHid; ++k) {
    float g = 0.0f;
    for (int j = 0; j < kMlpHid; ++j) g = fmaf(L.w[kOffW2 + j * kMlpHid + k], L.d2[s][j], g);
    L.d1[s][k] = h1[k] > 0.0f ? g : 0.0f;
  }
}

// Gradient contribution of one sub-batch (cnt samples) to parameter p.
__device__ float param_grad(const TrainLds& L, int p, int cnt) {
  float g = 0.0f;
  if (p < kOffB1) {
    const int j = p / kMlpIn, k = p % kMlpIn;
    for (int s = 0; s < cnt; ++s) g = fmaf(L.d1[s][j], L.x[s][k], g);
  } else if (p < kOffW2) {
    const int j = p - kOffB1;
    for (int s = 0; s < cnt; ++s) g += L.d1[s][j];
  } else if (p < kOffB2) {
    const int j = (p - kOffW2) / kMlpHid, k = (p - kOffW2) % kMlpHid;
    for (int s = 0; s < cnt; ++s) g = fmaf(L.d2[s][j], L.h1[s][k], g);
  } else if (p < kOffW3) {
    const int j = p - kOffB2;
    for (int s = 0; s < cnt; ++s) g += L.d2[s][j];
  } else if (p < kOffB3) {
    const int o = (p - kOffW3) / kMlpHid, k = (p - kOffW3) % kMlpHid;
    for (int s = 0; s < cnt; ++s) g = fmaf(L.dy[s][o], L.h2[s][k], g);
  } else {
    const int o = p - kOffB3;
    for (int s = 0; s < cnt; ++s) g += L.dy[s][o];
  }
  return g;
}

// Training (grad_out == nullptr) or one gradient evaluation of the first
// batch (grad_out != nullptr, weights unchanged).
__global__ __launch_bounds__(kTrainThreads) void mlp_train_kernel(
    const float* samples, int n, const int32_t* order, int epochs, int batch, float lr,
    float* w, float* m, float* v, float* loss_curve, float* grad_out, float* loss_out) {
  __shared__ TrainLds L;
  const int t = threadIdx.x;
  for (int p = t; p < kMlpParams; p += kTrainThreads) L.w[p] = w[p];
  __syncthreads();
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float b1t = 1.0f, b2t = 1.0f;
  for (int ep = 0; ep < epochs; ++ep) {
    double ep_loss = 0.0;
    for (int b0 = 0; b0 < n; b0 += batch) {
      const int B = min(batch, n - b0);
      const float invB = 1.0f / (float)B;
      float acc[kParamsPerThread];
      for (int q = 0; q < kParamsPerThread; ++q) acc[q] = 0.0f;
      for (int s0 = 0; s0 < B; s0 += kSub) {
        const int cnt = min(kSub, B - s0);
        if (t < cnt) {
          const int idx = order[(int64_t)ep * n + b0 + s0 + t];
          sample_pass(L, samples + (int64_t)idx * kSampleW, t, invB);
        }
        __syncthreads();
        for (int q = 0; q < kParamsPerThread; ++q) {
          const int p = t + q * kTrainThreads;
          if (p < kMlpParams) acc[q] += param_grad(L, p, cnt);
        }
        if (t == 0)
          for (int s = 0; s < cnt; ++s) ep_loss += (double)L.loss[s];
        __syncthreads();
      }
      if (grad_out) {
        for (int q = 0; q < kParamsPerThread; ++q) {
          const int p = t + q * kTrainThreads;
          if (p < kMlpParams) grad_out[p] = acc[q];
        }
        if (t == 0) *loss_out = (float)(ep_loss / (double)B);
        return;
      }
      b1t *= b1;
      b2t *= b2;
      for (int q = 0; q < kParamsPerThread; ++q) {
        const int p = t + q * kTrainThreads;
        if (p >= kMlpParams) continue;
        const float g = acc[q];
        const float mm = fmaf(b1, m[p], (1.0f - b1) * g);
        const float vv = fmaf(b2, v[p], (1.0f - b2) * g * g);
        m[p] = mm;
        v[p] = vv;
        const float mh = mm / (1.0f - b1t);
        const float vh = vv / (1.0f - b2t);
        L.w[p] -= lr * mh / (sqrtf(vh) + eps);
      }
      __syncthreads();
    }
    if (t == 0 && loss_curve) loss_curve[ep] = (float)(ep_loss / (double)n);
  }
  for (int p = t; p < kMlpParams; p += kTrainThreads) w[p] = L.w[p];
}

__global__ void mlp_forward_kernel(const float* w, const float* x, int n, float* y) {
  __shared__ __align__(16) float s_h[kForwardThreads / kWave][kMlpHid];
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= n) return;  // whole wave exits together
  float f[kMlpIn];
  for (int k = 0; k < kMlpIn; ++k) f[k] = x[(int64_t)i * kMlpIn + k];
  float y0, y1;
  mlp_forward_wave<kMlpHid>(w, w + kOffW2, f, y0, y1, s_h[threadIdx.x / kWave]);
  if (lane_id() == 0) {
    y[2 * (int64_t)i] = y0;
    y[2 * (int64_t)i + 1] = y1;
  }
}

struct DevBufs {
  std::vector<void*> ps;
  ~DevBufs() {
    for (void* p : ps) (void)rbfs::dev_free(p);
  }
  template <class T>
  hipError_t get(T** out, size_t count) {
    void* p = nullptr;
    hipError_t e = rbfs::dev_malloc(&p, sizeof(T) * (count > 0 ? count : 1));
    if (e == hipSuccess) {
      ps.push_back(p);
      *out = (T*)p;
    }
    return e;
  }
};

}  // namespace
}  // namespace rbfs

using rbfs::set_error;

#define ML_CHECK(x)                                                             \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      set_error(std::string(#x) + ": " + hipGetErrorString(e_));                \
      return e_ == hipErrorOutOfMemory ? RBFS_E_NOMEM : RBFS_E_DEVICE;          \
    }                                                                           \
  } while (0)

static int device_present() {
  int c = 0;
  if (hipGetDeviceCount(&c) != hipSuccess || c <= 0) {
    set_error("no HIP device");
    return RBFS_E_NODEV;
  }
  return 0;
}

extern "C" {

int rbfs_switch_load(const float* blob, int32_t n) {
  if (!blob || n != rbfs::kSwitchBlob) {
    set_error("rbfs_switch_load: expected " + std::to_string(rbfs::kSwitchBlob) + " floats");
    return RBFS_E_INVAL;
  }
  int rc = device_present();
  if (rc) return rc;
  int dev = 0;
  ML_CHECK(hipGetDevice(&dev));
  if (rbfs::s_switch_dev && rbfs::s_switch_device != dev) {
    (void)hipFree(rbfs::s_switch_dev);  // process lifetime
    rbfs::s_switch_dev = nullptr;
  }
  if (!rbfs::s_switch_dev) ML_CHECK(hipMalloc(&rbfs::s_switch_dev, sizeof(float) * n));
  rbfs::s_switch_device = dev;
  ML_CHECK(hipMemcpy(rbfs::s_switch_dev, blob, sizeof(float) * n, hipMemcpyHostToDevice));
  return RBFS_OK;
}

int rbfs_mlp_forward(const float* w, const float* x, int32_t n, float* y) {
  if (!w || !x || !y || n < 0) {
    set_error("rbfs_mlp_forward: bad arguments");
    return RBFS_E_INVAL;
  }
  int rc = device_present();
  if (rc) return rc;
  if (n == 0) return RBFS_OK;
  rbfs::DevBufs B;
  float *dw, *dx, *dy;
  ML_CHECK(B.get(&dw, rbfs::kMlpParams));
  ML_CHECK(B.get(&dx, (size_t)n * rbfs::kMlpIn));
  ML_CHECK(B.get(&dy, (size_t)n * rbfs::kMlpOut));
  ML_CHECK(hipMemcpy(dw, w, sizeof(float) * rbfs::kMlpParams, hipMemcpyHostToDevice));
  ML_CHECK(hipMemcpy(dx, x, sizeof(float) * n * rbfs::kMlpIn, hipMemcpyHostToDevice));
  const int per_block = rbfs::kForwardThreads / rbfs::kWave;  // one wave per sample
  hipLaunchKernelGGL(rbfs::mlp_forward_kernel, dim3((n + per_block - 1) / per_block),
                     dim3(rbfs::kForwardThreads), 0, 0, dw, dx, n, dy);
  ML_CHECK(hipGetLastError());
  ML_CHECK(hipMemcpy(y, dy, sizeof(float) * n * rbfs::kMlpOut, hipMemcpyDeviceToHost));
  return RBFS_OK;
}

static int train_common(const float* samples, int32_t n, const float* w_in,
                        const int32_t* order, int32_t epochs, int32_t batch, float lr,
                        float* w_out, float* loss_curve, float* grad, float* loss,
                        hipStream_t stream) {
  int rc = device_present();
  if (rc) return rc;
  rbfs::DevBufs B;
  float *ds, *dw, *dm, *dv, *dc = nullptr, *dg = nullptr, *dl = nullptr;
  int32_t* dord;
  ML_CHECK(B.get(&ds, (size_t)n * rbfs::kSampleW));
  ML_CHECK(B.get(&dw, rbfs::kMlpParams));
  ML_CHECK(B.get(&dm, rbfs::kMlpParams));
  ML_CHECK(B.get(&dv, rbfs::kMlpParams));
  ML_CHECK(B.get(&dord, (size_t)epochs * n));
  if (loss_curve) ML_CHECK(B.get(&dc, epochs));
  if (grad) {
    ML_CHECK(B.get(&dg, rbfs::kMlpParams));
    ML_CHECK(B.get(&dl, 1));
  }
  ML_CHECK(hipMemcpyAsync(ds, samples, sizeof(float) * n * rbfs::kSampleW,
                          hipMemcpyHostToDevice, stream));
  ML_CHECK(hipMemcpyAsync(dw, w_in, sizeof(float) * rbfs::kMlpParams, hipMemcpyHostToDevice,
                          stream));
  ML_CHECK(hipMemcpyAsync(dord, order, sizeof(int32_t) * epochs * n, hipMemcpyHostToDevice,
                          stream));
  ML_CHECK(hipMemsetAsync(dm, 0, sizeof(float) * rbfs::kMlpParams, stream));
  ML_CHECK(hipMemsetAsync(dv, 0, sizeof(float) * rbfs::kMlpParams, stream));
  hipLaunchKernelGGL(rbfs::mlp_train_kernel, dim3(1), dim3(rbfs::kTrainThreads), 0, stream, ds, n,
                     dord, epochs, batch, lr, dw, dm, dv, dc, dg, dl);
  ML_CHECK(hipGetLastError());
  if (w_out)
    ML_CHECK(hipMemcpyAsync(w_out, dw, sizeof(float) * rbfs::kMlpParams, hipMemcpyDeviceToHost,
                            stream));
  if (loss_curve)
    ML_CHECK(hipMemcpyAsync(loss_curve, dc, sizeof(float) * epochs, hipMemcpyDeviceToHost,
                            stream));
  if (grad) {
    ML_CHECK(hipMemcpyAsync(grad, dg, sizeof(float) * rbfs::kMlpParams, hipMemcpyDeviceToHost,
                            stream));
    ML_CHECK(hipMemcpyAsync(loss, dl, sizeof(float), hipMemcpyDeviceToHost, stream));
  }
  ML_CHECK(hipStreamSynchronize(stream));
  return RBFS_OK;
}

int rbfs_mlp_grad(const float* w, const float* samples, int32_t n, float* grad, float* loss) {
  if (!w || !samples || !grad || !loss || n < 1) {
    set_error("rbfs_mlp_grad: bad arguments");
    return RBFS_E_INVAL;
  }
  std::vector<int32_t> order(n);
  for (int32_t i = 0; i < n; ++i) order[i] = i;
  return train_common(samples, n, w, order.data(), 1, n, 0.0f, nullptr, nullptr, grad, loss,
                      nullptr);
}

int rbfs_mlp_backward(const float* w, const float* samples, int32_t n, float* grad,
                      float* loss) {
  return rbfs_mlp_grad(w, samples, n, grad, loss);
}

int rbfs_mlp_train(const float* samples, int32_t n, const float* w_init, const int32_t* order,
                   int32_t epochs, int32_t batch, float lr, float* w_out, float* loss_curve,
                   void* stream) {
  if (!samples || !w_init || !order || !w_out || n < 1 || epochs < 1 || batch < 1 ||
      !(lr > 0.0f)) {
    set_error("rbfs_mlp_train: bad arguments");
    return RBFS_E_INVAL;
  }
  for (int64_t i = 0; i < (int64_t)epochs * n; ++i) {
    if (order[i] < 0 || order[i] >= n) {
      set_error("rbfs_mlp_train: order entry out of range");
      return RBFS_E_RANGE;
    }
  }
  return train_common(samples, n, w_init, order, epochs, batch, lr, w_out, loss_curve, nullptr,
                      nullptr, (hipStream_t)stream);
}

// Training samples (defined with the search API): per root and level, the
// cost of each direction from that level to the end of the search.  Row
// layout (11 floats): features[8], ln(us top-down), ln(us bottom-up), level.
int rbfs_collect_level_samples(rbfs_graph_t* h, const int32_t* roots, int32_t k, int32_t reps,
                               int32_t alpha, int32_t beta, float* out, int32_t cap,
                               int32_t* count, void* stream);

}  // extern "C"
