// Conjugate gradients on the device, every product through a plan of the
// speculative segmented sum.
//
// Section 1 of the paper gives the reason for computing on CSR as it arrives:
// an iterative solver multiplies the same matrix a few hundred times, and a
// conversion to another format would cost about as much as the solve.  This
// file is that use: Hestenes and Stiefel's iteration for a symmetric positive
// definite A, with the vector steps and dot products in kernels of their own,
// so that an iteration is the two stages of the product plus three short
// launches and the host never waits inside the loop:
//
//   cg_pq         partial sums of p.q, one per workgroup
//   cg_residual   alpha = (r.r) / (p.q); r -= alpha q; partial sums of the
//                 new r.r
//   cg_direction  beta = (r.r)_new / (r.r); x += alpha p; p = r + beta p;
//                 stores (r.r)_new
//
// x moves in the last kernel, beside p, because that kernel reads p anyway:
// the three kernels then stream 10 vectors of m doubles per iteration
// instead of 11.
//
// Every workgroup of cg_residual and cg_direction adds up all the partial sums
// itself, in the same fixed order, so each holds the same scalar bit for bit
// without a grid-wide wait.  The scalars live in a small work array:
//   [0] r.r of the current residual (read by cg_residual, written by
//       workgroup 0 of cg_direction)
//   [1] r.r before the step under way (written by workgroup 0 of
//       cg_residual, read by cg_direction)
//   [2] b.b
//   [3] alpha of the step under way (written by workgroup 0 of cg_residual,
//       read by cg_direction)
//   [kPartA ...) the per-workgroup partial sums of p.q (at the start: r.r)
//   [kPartB ...) the per-workgroup partial sums of the new r.r (start: b.b)
// No kernel writes a word that another workgroup of the same launch reads.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "sss.h"

namespace {

constexpr int kWave = 64;
constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;  // workgroups of a vector kernel: partial sums per dot product
constexpr int kRho = 0, kRhoPrev = 1, kBB = 2, kAlpha = 3;
constexpr int kPartA = 8;
constexpr int kPartB = kPartA + kMaxBlocks;
constexpr int kWorkDoubles = kPartB + kMaxBlocks;

thread_local hipError_t g_cg_hip = hipSuccess;

// sum over the wavefront by butterfly: every lane ends with the same bits
// (each step adds the same two values in every lane of a pair)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// sum over the workgroup, the same bits in every thread
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = v;
  __syncthreads();
  const double s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();  // lds is reused by the next sum
  return s;
}

// the sum of the nblk partial sums, the same in every workgroup
__device__ __forceinline__ double sum_partials(const double *part, int nblk, double *lds) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kThreads) v += part[i];
  return block_sum(v, lds);
}

__device__ __forceinline__ int64_t first_index() { return (int64_t)blockIdx.x * kThreads + threadIdx.x; }
__device__ __forceinline__ int64_t grid_stride() { return (int64_t)gridDim.x * kThreads; }
// each thread issues the loads of kU elements, a grid stride apart, before
// it uses any of them: kU times the loads in flight of a plain grid-stride
// loop (0.95 us less per iteration over the three kernels at 1M rows)
constexpr int kU = 4;

// r = b - q, p = r; partial sums of r.r and b.b
__global__ __launch_bounds__(kThreads) void cg_start(const double *__restrict__ b, const double *__restrict__ q,
                                                     double *__restrict__ r, double *__restrict__ p,
                                                     double *__restrict__ work, int64_t m) {
  __shared__ double lds[kThreads / kWave];
  double rr = 0.0, bb = 0.0;
  for (int64_t i = first_index(); i < m; i += grid_stride()) {
    const double bi = b[i];
    const double ri = bi - q[i];
    r[i] = ri;
    p[i] = ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  rr = block_sum(rr, lds);
  bb = block_sum(bb, lds);
  if (threadIdx.x == 0) {
    work[kPartA + blockIdx.x] = rr;
    work[kPartB + blockIdx.x] = bb;
  }
}

// one workgroup: r.r and b.b from the start's partial sums
__global__ __launch_bounds__(kThreads) void cg_start_sums(double *__restrict__ work, int nblk) {
  __shared__ double lds[kThreads / kWave];
  const double rr = sum_partials(work + kPartA, nblk, lds);
  const double bb = sum_partials(work + kPartB, nblk, lds);
  if (threadIdx.x == 0) {
    work[kRho] = rr;
    work[kRhoPrev] = rr;
    work[kBB] = bb;
    work[kAlpha] = 0.0;
  }
}

// partial sums of p.q
__global__ __launch_bounds__(kThreads) void cg_pq(const double *__restrict__ p, const double *__restrict__ q,
                                                  double *__restrict__ work, int64_t m) {
  __shared__ double lds[kThreads / kWave];
  double s = 0.0;
  const int64_t gs = grid_stride();
  for (int64_t base = first_index(); base < m; base += kU * gs) {
    double pv[kU], qv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + u * gs;
      pv[u] = i < m ? p[i] : 0.0;
      qv[u] = i < m ? q[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) s += pv[u] * qv[u];
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) work[kPartA + blockIdx.x] = s;
}

// alpha = (r.r) / (p.q); r -= alpha q; partial sums of the new r.r
__global__ __launch_bounds__(kThreads) void cg_residual(const double *__restrict__ q, double *__restrict__ r,
                                                        double *__restrict__ work, int64_t m, int nblk) {
  __shared__ double lds[kThreads / kWave];
  const double pq = sum_partials(work + kPartA, nblk, lds);
  const double rho = work[kRho];
  const double alpha = pq != 0.0 ? rho / pq : 0.0;
  double rr = 0.0;
  const int64_t gs = grid_stride();
  for (int64_t base = first_index(); base < m; base += kU * gs) {
    double rv[kU], qv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + u * gs;
      rv[u] = i < m ? r[i] : 0.0;
      qv[u] = i < m ? q[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + u * gs;
      const double ri = rv[u] - alpha * qv[u];
      if (i < m) r[i] = ri;
      rr += ri * ri;
    }
  }
  rr = block_sum(rr, lds);
  if (threadIdx.x == 0) {
    work[kPartB + blockIdx.x] = rr;
    if (blockIdx.x == 0) {
      work[kRhoPrev] = rho;
      work[kAlpha] = alpha;
    }
  }
}

// beta = (r.r)_new / (r.r); x += alpha p; p = r + beta p; stores (r.r)_new
__global__ __launch_bounds__(kThreads) void cg_direction(const double *__restrict__ r, double *__restrict__ p,
                                                         double *__restrict__ x, double *__restrict__ work,
                                                         int64_t m, int nblk) {
  __shared__ double lds[kThreads / kWave];
  const double rho_new = sum_partials(work + kPartB, nblk, lds);
  const double rho = work[kRhoPrev];
  const double alpha = work[kAlpha];
  const double beta = rho != 0.0 ? rho_new / rho : 0.0;
  const int64_t gs = grid_stride();
  for (int64_t base = first_index(); base < m; base += kU * gs) {
    double pv[kU], xv[kU], rv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + u * gs;
      pv[u] = i < m ? p[i] : 0.0;
      xv[u] = i < m ? x[i] : 0.0;
      rv[u] = i < m ? r[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + u * gs;
      if (i < m) {
        x[i] = xv[u] + alpha * pv[u];
        p[i] = rv[u] + beta * pv[u];
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) work[kRho] = rho_new;
}

int vector_blocks(int64_t m) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxBlocks, (m + kThreads * kU - 1) / (kThreads * kU)));
}

bool aligned8(const void *ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 7) == 0; }

// the plan's m, after the checks every CG call makes
int check_plan(sss_plan p, int64_t *m) {
  int64_t n = 0;
  sss_dtype dt = SSS_F64;
  const int rc = sss_plan_shape(p, m, &n, nullptr, &dt);
  if (rc != SSS_OK) return rc;
  if (dt != SSS_F64) return SSS_ERR_UNSUPPORTED;
  if (*m != n) return SSS_ERR_INVALID_VALUE;
  return SSS_OK;
}

int launch_status() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_cg_hip = e;
    return SSS_ERR_HIP;
  }
  return SSS_OK;
}

}  // namespace

extern "C" {

int sss_cg_workspace_size(size_t *bytes) {
  if (!bytes) return SSS_ERR_INVALID_VALUE;
  *bytes = sizeof(double) * kWorkDoubles;
  return SSS_OK;
}

int sss_cg_start(sss_plan p, const int32_t *row_ptr, const int32_t *col, const double *val, const double *b,
                 const double *x, double *r, double *dir, double *q, void *work, void *stream) {
  int64_t m = 0;
  int rc = check_plan(p, &m);
  if (rc != SSS_OK) return rc;
  if (!work || !aligned8(work)) return SSS_ERR_INVALID_VALUE;
  if (m > 0 && (!b || !x || !r || !dir || !q)) return SSS_ERR_INVALID_VALUE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *w = static_cast<double *>(work);
  int nblk = 0;
  if (m > 0) {
    rc = sss_csr_spmv_execute(p, row_ptr, col, val, x, q, stream);
    if (rc != SSS_OK) return rc;
    nblk = vector_blocks(m);
    hipLaunchKernelGGL(cg_start, dim3(nblk), dim3(kThreads), 0, s, b, q, r, dir, w, m);
    if ((rc = launch_status()) != SSS_OK) return rc;
  }
  hipLaunchKernelGGL(cg_start_sums, dim3(1), dim3(kThreads), 0, s, w, nblk);
  return launch_status();
}

int sss_cg_iterate(sss_plan p, const int32_t *row_ptr, const int32_t *col, const double *val, double *x,
                   double *r, double *dir, double *q, void *work, int iterations, void *stream) {
  int64_t m = 0;
  int rc = check_plan(p, &m);
  if (rc != SSS_OK) return rc;
  if (iterations < 0 || !work || !aligned8(work)) return SSS_ERR_INVALID_VALUE;
  if (m == 0 || iterations == 0) return SSS_OK;
  if (!x || !r || !dir || !q) return SSS_ERR_INVALID_VALUE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *w = static_cast<double *>(work);
  const int nblk = vector_blocks(m);
  for (int it = 0; it < iterations; ++it) {
    rc = sss_csr_spmv_execute(p, row_ptr, col, val, dir, q, stream);
    if (rc != SSS_OK) return rc;
    hipLaunchKernelGGL(cg_pq, dim3(nblk), dim3(kThreads), 0, s, dir, q, w, m);
    hipLaunchKernelGGL(cg_residual, dim3(nblk), dim3(kThreads), 0, s, q, r, w, m, nblk);
    hipLaunchKernelGGL(cg_direction, dim3(nblk), dim3(kThreads), 0, s, r, dir, x, w, m, nblk);
    if ((rc = launch_status()) != SSS_OK) return rc;
  }
  return SSS_OK;
}

const char *sss_cg_last_hip_error(void) { return hipGetErrorString(g_cg_hip); }

}  // extern "C"
