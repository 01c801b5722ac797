// Parameter selection for the speculative segmented sum SpMV on gfx950.
//
// The paper fixes T to the SIMD width and picks W (nonzeros per lane) and S
// (tiles per thread-bunch) empirically per processor (Section 3.4, Table 3;
// Section 4.5 sweeps both).  Here the choice is per matrix:
//   * a grid autotuner times every (W, S) class of the parameter grid on the
//     caller's matrix and keeps the fastest;
//   * a small network (8 -> 64 -> 64 -> 12, ReLU) maps matrix features to a
//     class; it is trained on the autotuner's timings by the forward,
//     backward and Adam kernels below, and runs inference with the same
//     forward kernels.
// Features come from one pass over row_ptr on the device.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "sss.h"

namespace {

constexpr int kIn = SSS_N_FEATURES, kHid = SSS_MLP_HIDDEN, kOut = SSS_N_CLASSES;
constexpr int kFeatBlocks = 256, kFeatThreads = 256;
constexpr int kTrials = 5;  // autotuner: timed rounds over the classes

thread_local hipError_t g_sel_hip = hipSuccess;

#define SEL_HIP(call)                         \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) {                   \
      g_sel_hip = e_;                         \
      return SSS_ERR_HIP;                     \
    }                                         \
  } while (0)

// (W, S) of each class: W in {4, 8, 16} x S in {1, 2, 4, 8}
constexpr int kClassW[kOut] = {4, 4, 4, 4, 8, 8, 8, 8, 16, 16, 16, 16};
constexpr int kClassS[kOut] = {1, 2, 4, 8, 1, 2, 4, 8, 1, 2, 4, 8};

// ---------------------------------------------------------------- features

// Per block: sum of row lengths, sum of squares, max length, empty rows, in
// a fixed reduction order (per thread over a grid stride, then an LDS tree).
__global__ __launch_bounds__(kFeatThreads) void sss_row_stats(const int32_t *__restrict__ rp, int64_t m,
                                                              double *__restrict__ part) {
  __shared__ double s1[kFeatThreads], s2[kFeatThreads];
  __shared__ long long smax[kFeatThreads], semp[kFeatThreads];
  double a = 0.0, b = 0.0;
  long long mx = 0, em = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    const long long L = (long long)rp[r + 1] - (long long)rp[r];
    a += (double)L;
    b += (double)L * (double)L;
    mx = L > mx ? L : mx;
    em += (L == 0);
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  smax[threadIdx.x] = mx;
  semp[threadIdx.x] = em;
  __syncthreads();
  for (int d = blockDim.x / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
      s1[threadIdx.x] += s1[threadIdx.x + d];
      s2[threadIdx.x] += s2[threadIdx.x + d];
      smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + d]);
      semp[threadIdx.x] += semp[threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = s1[0];
    part[4 * blockIdx.x + 1] = s2[0];
    part[4 * blockIdx.x + 2] = (double)smax[0];
    part[4 * blockIdx.x + 3] = (double)semp[0];
  }
}

// The per-block partial statistics: one array per device in the code object
// (no allocation per call); calls are serialised by a mutex and each waits
// for its stream before it returns.
__device__ double feat_part[4 * kFeatBlocks];
std::mutex g_feat_mu;
double *g_feat_ptr[64] = {};

// ---------------------------------------------------------------- network

// Y[n][o] = act(sum_i X[n][i] W[i][o] + b[o]); one thread per output.
template <bool RELU>
__global__ void mlp_dense_fwd(const float *__restrict__ X, const float *__restrict__ Wt, const float *__restrict__ bias,
                              float *__restrict__ Y, int N, int I, int O) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * O) return;
  const int n = (int)(t / O), o = (int)(t % O);
  float acc = bias[o];
  for (int i = 0; i < I; ++i) acc = fmaf(X[(int64_t)n * I + i], Wt[i * O + o], acc);
  Y[t] = RELU ? fmaxf(acc, 0.f) : acc;
}

// softmax cross-entropy against target distributions Q: dZ = (softmax(Z) - Q)/N
// and the per-sample loss; one thread per sample.
__global__ void mlp_softmax_ce(const float *__restrict__ Z, const float *__restrict__ Q, float *__restrict__ dZ,
                               float *__restrict__ loss, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const float *z = Z + (int64_t)n * kOut;
  float mx = z[0];
  for (int c = 1; c < kOut; ++c) mx = fmaxf(mx, z[c]);
  float se = 0.f;
  for (int c = 0; c < kOut; ++c) se += expf(z[c] - mx);
  const float lse = mx + logf(se);
  float l = 0.f;
  for (int c = 0; c < kOut; ++c) {
    const float q = Q[(int64_t)n * kOut + c];
    dZ[(int64_t)n * kOut + c] = (expf(z[c] - lse) - q) / (float)N;
    l -= q * (z[c] - lse);
  }
  if (loss) loss[n] = l;
}

// dW[i][o] = sum_n X[n][i] dZ[n][o]; db[o] = sum_n dZ[n][o]: one thread per
// weight (and per bias), summing over n in order.
__global__ void mlp_dense_bwd_w(const float *__restrict__ X, const float *__restrict__ dZ, float *__restrict__ dW,
                                float *__restrict__ db, int N, int I, int O) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < I * O) {
    const int i = t / O, o = t % O;
    float acc = 0.f;
    for (int n = 0; n < N; ++n) acc = fmaf(X[(int64_t)n * I + i], dZ[(int64_t)n * O + o], acc);
    dW[t] = acc;
  } else if (t < I * O + O) {
    const int o = t - I * O;
    float acc = 0.f;
    for (int n = 0; n < N; ++n) acc += dZ[(int64_t)n * O + o];
    db[o] = acc;
  }
}

// dH[n][i] = (sum_o dZ[n][o] W[i][o]) * (H[n][i] > 0); one thread per entry.
__global__ void mlp_dense_bwd_x(const float *__restrict__ dZ, const float *__restrict__ Wt,
                                const float *__restrict__ H, float *__restrict__ dH, int N, int I, int O) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * I) return;
  const int n = (int)(t / I), i = (int)(t % I);
  float acc = 0.f;
  for (int o = 0; o < O; ++o) acc = fmaf(dZ[(int64_t)n * O + o], Wt[i * O + o], acc);
  dH[t] = H[t] > 0.f ? acc : 0.f;
}

__global__ void mlp_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                         float *__restrict__ m2, int n, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  p[i] -= lr * (a / bc1) / (sqrtf(v / bc2) + eps);
}

// offsets of the packed parameter blocks
constexpr int oW1 = 0, ob1 = oW1 + kIn * kHid, oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid, oW3 = ob2 + kHid,
              ob3 = oW3 + kHid * kOut, kParams = ob3 + kOut;
static_assert(kParams == SSS_MLP_PARAMS, "parameter count");

unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int forward_launch(const float *P, const float *X, int N, float *H1, float *H2, float *Z, hipStream_t s) {
  hipLaunchKernelGGL(mlp_dense_fwd<true>, dim3(nblk((int64_t)N * kHid, 256)), dim3(256), 0, s, X, P + oW1, P + ob1,
                     H1, N, kIn, kHid);
  hipLaunchKernelGGL(mlp_dense_fwd<true>, dim3(nblk((int64_t)N * kHid, 256)), dim3(256), 0, s, H1, P + oW2, P + ob2,
                     H2, N, kHid, kHid);
  hipLaunchKernelGGL(mlp_dense_fwd<false>, dim3(nblk((int64_t)N * kOut, 256)), dim3(256), 0, s, H2, P + oW3,
                     P + ob3, Z, N, kHid, kOut);
  SEL_HIP(hipGetLastError());
  return SSS_OK;
}

// ---------------------------------------------------------------- selector state

struct SelectorState {
  bool loaded = false;
  float mean[kIn], stdv[kIn];
  float *d_params = nullptr;  // kParams
  float *d_work = nullptr;    // X (kIn), H1, H2 (kHid each), Z (kOut)
  int device = -1;
};
std::mutex g_sel_mu;
SelectorState g_sel[64];

// The autotuners' timing protocol.  Two warm-up runs of every candidate, then
// kTrials rounds over the candidates in turn (a clock ramp or any other
// transient lands on one trial of one candidate, which the median drops);
// each trial is `reps` back-to-back runs between two events on `s`, i.e. the
// device's time per run, not the host's launch latency.  med[c] = the median
// trial's microseconds per run of candidate c.
template <typename Run>
int time_interleaved(int n, const Run &run, int reps, hipStream_t s, float *med) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = SSS_OK;
  if (hipEventCreate(&e0) != hipSuccess) rc = SSS_ERR_HIP;
  if (rc == SSS_OK && hipEventCreate(&e1) != hipSuccess) rc = SSS_ERR_HIP;
  for (int c = 0; c < n && rc == SSS_OK; ++c)
    for (int k = 0; k < 2 && rc == SSS_OK; ++k) rc = run(c);
  std::vector<std::vector<float>> t((size_t)n);
  for (int r = 0; r < kTrials && rc == SSS_OK; ++r) {
    for (int c = 0; c < n && rc == SSS_OK; ++c) {
      hipError_t e = hipEventRecord(e0, s);
      for (int k = 0; k < reps && rc == SSS_OK && e == hipSuccess; ++k) rc = run(c);
      if (rc == SSS_OK && e == hipSuccess) e = hipEventRecord(e1, s);
      if (rc == SSS_OK && e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (rc == SSS_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) { g_sel_hip = e; rc = SSS_ERR_HIP; }
      t[(size_t)c].push_back(ms * 1000.f / (float)reps);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc != SSS_OK) return rc;
  for (int c = 0; c < n; ++c) {
    std::sort(t[(size_t)c].begin(), t[(size_t)c].end());
    med[c] = t[(size_t)c][t[(size_t)c].size() / 2];
  }
  return SSS_OK;
}

int argmin(const float *v, int n) {
  int best = 0;
  for (int c = 1; c < n; ++c)
    if (v[c] < v[best]) best = c;
  return best;
}

}  // namespace

extern "C" {

int sss_class_params(int cls, int *W, int *S) {
  if (cls < 0 || cls >= kOut) return SSS_ERR_INVALID_VALUE;
  if (W) *W = kClassW[cls];
  if (S) *S = kClassS[cls];
  return SSS_OK;
}

int sss_csr_features(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, sss_dtype dt, void *stream,
                     float *feats) {
  if (m < 0 || n < 0 || nnz < 0 || !feats || (m > 0 && !row_ptr)) return SSS_ERR_INVALID_VALUE;
  double sum = 0, sq = 0, mx = 0, em = 0;
  if (m > 0) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    SEL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return SSS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_feat_mu);
    if (!g_feat_ptr[dev]) {
      void *ptr = nullptr;
      SEL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(feat_part)));
      g_feat_ptr[dev] = static_cast<double *>(ptr);
    }
    double *d_part = g_feat_ptr[dev];
    std::vector<double> part(4 * kFeatBlocks);
    hipLaunchKernelGGL(sss_row_stats, dim3(kFeatBlocks), dim3(kFeatThreads), 0, s, row_ptr, m, d_part);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(part.data(), d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { g_sel_hip = e; return SSS_ERR_HIP; }
    for (int b = 0; b < kFeatBlocks; ++b) {
      sum += part[4 * b];
      sq += part[4 * b + 1];
      mx = std::max(mx, part[4 * b + 2]);
      em += part[4 * b + 3];
    }
  }
  const double mean = m > 0 ? sum / (double)m : 0.0;
  const double var = m > 0 ? std::max(0.0, sq / (double)m - mean * mean) : 0.0;
  feats[0] = (float)std::log2((double)m + 1.0);
  feats[1] = (float)std::log2((double)n + 1.0);
  feats[2] = (float)std::log2((double)nnz + 1.0);
  feats[3] = (float)std::log2(1.0 + mean);
  feats[4] = (float)std::log2(1.0 + var);
  feats[5] = (float)std::log2(1.0 + mx);
  feats[6] = m > 0 ? (float)(em / (double)m) : 0.f;
  feats[7] = dt == SSS_F64 ? 8.f : (dt == SSS_F32 ? 4.f : 2.f);
  return SSS_OK;
}

int sss_mlp_forward(const float *params, const float *X, int N, float *H1, float *H2, float *Z, void *stream) {
  if (N < 0 || (N > 0 && (!params || !X || !H1 || !H2 || !Z))) return SSS_ERR_INVALID_VALUE;
  if (N == 0) return SSS_OK;
  return forward_launch(params, X, N, H1, H2, Z, static_cast<hipStream_t>(stream));
}

int sss_mlp_backward(const float *params, const float *X, const float *H1, const float *H2, const float *Z,
                     const float *Q, int N, float *grad, float *loss, float *work, void *stream) {
  if (N <= 0 || !params || !X || !H1 || !H2 || !Z || !Q || !grad || !work) return SSS_ERR_INVALID_VALUE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *dZ = work;                              // N x 12
  float *dH2 = dZ + (int64_t)N * kOut;           // N x 64
  float *dH1 = dH2 + (int64_t)N * kHid;          // N x 64
  hipLaunchKernelGGL(mlp_softmax_ce, dim3(nblk(N, 256)), dim3(256), 0, s, Z, Q, dZ, loss, N);
  hipLaunchKernelGGL(mlp_dense_bwd_w, dim3(nblk(kHid * kOut + kOut, 256)), dim3(256), 0, s, H2, dZ, grad + oW3,
                     grad + ob3, N, kHid, kOut);
  hipLaunchKernelGGL(mlp_dense_bwd_x, dim3(nblk((int64_t)N * kHid, 256)), dim3(256), 0, s, dZ, params + oW3, H2, dH2,
                     N, kHid, kOut);
  hipLaunchKernelGGL(mlp_dense_bwd_w, dim3(nblk(kHid * kHid + kHid, 256)), dim3(256), 0, s, H1, dH2, grad + oW2,
                     grad + ob2, N, kHid, kHid);
  hipLaunchKernelGGL(mlp_dense_bwd_x, dim3(nblk((int64_t)N * kHid, 256)), dim3(256), 0, s, dH2, params + oW2, H1, dH1,
                     N, kHid, kHid);
  hipLaunchKernelGGL(mlp_dense_bwd_w, dim3(nblk(kIn * kHid + kHid, 256)), dim3(256), 0, s, X, dH1, grad + oW1,
                     grad + ob1, N, kIn, kHid);
  SEL_HIP(hipGetLastError());
  return SSS_OK;
}

int sss_mlp_adam(float *params, const float *grad, float *m1, float *m2, int n, int step, float lr, float beta1,
                 float beta2, float eps, void *stream) {
  if (n < 0 || step < 1 || (n > 0 && (!params || !grad || !m1 || !m2))) return SSS_ERR_INVALID_VALUE;
  if (n == 0) return SSS_OK;
  const float bc1 = 1.f - std::pow(beta1, (float)step), bc2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(mlp_adam, dim3(nblk(n, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), params, grad, m1,
                     m2, n, lr, beta1, beta2, eps, bc1, bc2);
  SEL_HIP(hipGetLastError());
  return SSS_OK;
}

int sss_selector_set(const float *params, const float *mean, const float *stdv) {
  if (!params || !mean || !stdv) return SSS_ERR_INVALID_VALUE;
  int dev = 0;
  SEL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SSS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_sel_mu);
  SelectorState &st = g_sel[dev];
  if (!st.d_params) {
    SEL_HIP(hipMalloc(&st.d_params, sizeof(float) * kParams));
    SEL_HIP(hipMalloc(&st.d_work, sizeof(float) * (kIn + 2 * kHid + kOut)));
  }
  SEL_HIP(hipMemcpy(st.d_params, params, sizeof(float) * kParams, hipMemcpyHostToDevice));
  std::memcpy(st.mean, mean, sizeof(st.mean));
  std::memcpy(st.stdv, stdv, sizeof(st.stdv));
  st.loaded = true;
  st.device = dev;
  return SSS_OK;
}

int sss_selector_scores(const float *feats, float *logits) {
  if (!feats || !logits) return SSS_ERR_INVALID_VALUE;
  int dev = 0;
  SEL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SSS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_sel_mu);
  SelectorState &st = g_sel[dev];
  if (!st.loaded) return SSS_ERR_UNSUPPORTED;
  float x[kIn];
  for (int i = 0; i < kIn; ++i) x[i] = (feats[i] - st.mean[i]) / (st.stdv[i] > 0.f ? st.stdv[i] : 1.f);
  float *dX = st.d_work, *dH1 = dX + kIn, *dH2 = dH1 + kHid, *dZ = dH2 + kHid;
  SEL_HIP(hipMemcpy(dX, x, sizeof(x), hipMemcpyHostToDevice));
  const int rc = forward_launch(st.d_params, dX, 1, dH1, dH2, dZ, nullptr);
  if (rc != SSS_OK) return rc;
  SEL_HIP(hipMemcpy(logits, dZ, sizeof(float) * kOut, hipMemcpyDeviceToHost));
  return SSS_OK;
}

int sss_selector_predict(const float *feats, int *cls) {
  if (!feats || !cls) return SSS_ERR_INVALID_VALUE;
  int dev = 0;
  SEL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SSS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_sel_mu);
  SelectorState &st = g_sel[dev];
  if (!st.loaded) return SSS_ERR_UNSUPPORTED;
  float x[kIn], z[kOut];
  for (int i = 0; i < kIn; ++i) x[i] = (feats[i] - st.mean[i]) / (st.stdv[i] > 0.f ? st.stdv[i] : 1.f);
  float *dX = st.d_work, *dH1 = dX + kIn, *dH2 = dH1 + kHid, *dZ = dH2 + kHid;
  SEL_HIP(hipMemcpy(dX, x, sizeof(x), hipMemcpyHostToDevice));
  const int rc = forward_launch(st.d_params, dX, 1, dH1, dH2, dZ, nullptr);
  if (rc != SSS_OK) return rc;
  SEL_HIP(hipMemcpy(z, dZ, sizeof(z), hipMemcpyDeviceToHost));
  int best = 0;
  for (int c = 1; c < kOut; ++c)
    if (z[c] > z[best]) best = c;
  *cls = best;
  return SSS_OK;
}

int sss_selector_loaded(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  std::lock_guard<std::mutex> lk(g_sel_mu);
  return g_sel[dev].loaded ? 1 : 0;
}

int sss_csr_spmv_autotune(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                          const void *val, const void *x, void *y, sss_dtype dt, int reps, void *stream,
                          float *class_us, int *best_class) {
  if (reps < 1 || !best_class) return SSS_ERR_INVALID_VALUE;
  sss_plan plans[kOut] = {};
  int rc = SSS_OK;
  // the classes are timed as they run for this matrix: rows bound at plan time
  const int bind = (m > 0 && nnz > 0) ? 1 : 0;
  for (int c = 0; c < kOut && rc == SSS_OK; ++c) {
    sss_plan_opts o = {SSS_MODE_FIXED, kClassW[c], kClassS[c], 0, 0, bind};
    rc = sss_csr_spmv_plan_create(m, n, nnz, row_ptr, dt, &o, stream, &plans[c]);
  }
  float med[kOut];
  if (rc == SSS_OK)
    rc = time_interleaved(
        kOut, [&](int c) { return sss_csr_spmv_execute(plans[c], row_ptr, col, val, x, y, stream); }, reps,
        static_cast<hipStream_t>(stream), med);
  for (int c = 0; c < kOut; ++c) {
    const int drc = sss_plan_destroy(plans[c]);
    if (rc == SSS_OK) rc = drc;
  }
  if (rc != SSS_OK) return rc;
  *best_class = argmin(med, kOut);
  if (class_us) std::memcpy(class_us, med, sizeof(med));
  return SSS_OK;
}

int sss_csr_spmv_plan_create_grid(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                                  const void *val, const void *x, void *y, sss_dtype dt, int reps, void *stream,
                                  sss_plan *out) {
  if (!out) return SSS_ERR_INVALID_VALUE;
  *out = nullptr;
  sss_plan_opts o = {SSS_MODE_FIXED, 0, 0, 0, 0, 0};
  if (m > 0 && nnz > 0) {
    int best = 0;
    const int rc = sss_csr_spmv_autotune(m, n, nnz, row_ptr, col, val, x, y, dt, reps, stream, nullptr, &best);
    if (rc != SSS_OK) return rc;
    o.W = kClassW[best];
    o.S = kClassS[best];
    o.bind_rows = 1;
  }
  return sss_csr_spmv_plan_create(m, n, nnz, row_ptr, dt, &o, stream, out);
}

int sss_batch_plan_create_grid(int count, const sss_csr_desc *mats, sss_dtype dt, int reps, void *stream,
                               float *class_us, int *best_class, sss_plan *out) {
  if (!out || reps < 1 || count < 0 || (count > 0 && !mats)) return SSS_ERR_INVALID_VALUE;
  *out = nullptr;
  // every matrix takes the class's S: per-matrix S in the descriptors is
  // ignored here
  std::vector<sss_csr_desc> d(mats, mats + count);
  for (auto &e : d) e.S = 0;
  sss_plan plans[kOut] = {};
  int rc = SSS_OK;
  for (int c = 0; c < kOut && rc == SSS_OK; ++c) {
    sss_plan_opts o = {SSS_MODE_FIXED, kClassW[c], kClassS[c], 0, 0};
    rc = sss_batch_plan_create(count, d.data(), dt, &o, stream, &plans[c]);
  }
  float med[kOut];
  if (rc == SSS_OK)
    rc = time_interleaved(kOut, [&](int c) { return sss_batch_execute(plans[c], stream); }, reps,
                          static_cast<hipStream_t>(stream), med);
  const int best = rc == SSS_OK ? argmin(med, kOut) : -1;
  for (int c = 0; c < kOut; ++c) {
    if (c == best) continue;
    const int drc = sss_plan_destroy(plans[c]);
    if (rc == SSS_OK) rc = drc;
  }
  if (rc != SSS_OK) {
    if (best >= 0) (void)sss_plan_destroy(plans[best]);
    return rc;
  }
  if (class_us) std::memcpy(class_us, med, sizeof(med));
  if (best_class) *best_class = best;
  *out = plans[best];
  return SSS_OK;
}

const char *sss_selector_last_hip_error(void) { return hipGetErrorString(g_sel_hip); }

}  // extern "C"
