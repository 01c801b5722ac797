// Row-wise CSR SpMV comparators for gfx950 -- NOT the speculative method.
//
// The paper measures the speculative segmented sum against row-wise GPU
// kernels (Section 4.3): "CSR-scalar", one thread per row, and "CSR-vector",
// one SIMD unit per row with a reduction across its lanes.  Section 2.1
// explains why they lose on irregular matrices: a thread or wavefront that
// owns a long row serialises it while its neighbours idle, and short rows
// leave lanes idle in the vector form.  These kernels are written here from
// that description so that the comparison can be repeated on MI355X.  One
// kernel covers both: L lanes per row, L = 1 (scalar) ... 64 (a whole
// wavefront per row); the lanes of a row stride over it and then reduce by
// shuffles within their aligned group of L lanes.  Plain (uncompensated)
// sums in the value type's accumulator: double for F64, float for F32/BF16.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "sss.h"

namespace {

constexpr int kWave = 64;
constexpr int kThreads = 256;

thread_local hipError_t g_rw_hip = hipSuccess;

template <int DT> struct RowT;
template <> struct RowT<SSS_F64> { using val_t = double;   using x_t = double; using acc_t = double; };
template <> struct RowT<SSS_F32> { using val_t = float;    using x_t = float;  using acc_t = float; };
template <> struct RowT<SSS_BF16>{ using val_t = uint16_t; using x_t = float;  using acc_t = float; };

__device__ __forceinline__ double rw_val(const double *v, int64_t k) { return v[k]; }
__device__ __forceinline__ float rw_val(const float *v, int64_t k) { return v[k]; }
__device__ __forceinline__ float rw_val(const uint16_t *v, int64_t k) { return __uint_as_float((uint32_t)v[k] << 16); }

template <int DT, int L>
__global__ __launch_bounds__(kThreads) void sss_rowwise(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       const void *__restrict__ val_, const void *__restrict__ x_,
                                                       void *__restrict__ y_, int64_t m) {
  using val_t = typename RowT<DT>::val_t;
  using x_t = typename RowT<DT>::x_t;
  using acc_t = typename RowT<DT>::acc_t;
  const val_t *__restrict__ val = static_cast<const val_t *>(val_);
  const x_t *__restrict__ x = static_cast<const x_t *>(x_);
  x_t *__restrict__ y = static_cast<x_t *>(y_);
  const int sub = threadIdx.x % L;  // lane within the row's group
  const int64_t groups = (int64_t)gridDim.x * (kThreads / L);
  for (int64_t row = (int64_t)blockIdx.x * (kThreads / L) + threadIdx.x / L;; row += groups) {
    // every lane of a wavefront runs the same number of iterations (the
    // shuffles below need the whole wavefront): stop once the wavefront's
    // first row is past the end
    const int64_t first = __shfl(row, 0, kWave);
    if (first >= m) break;
    acc_t s = 0;
    if (row < m) {
      const int64_t lo = rp[row], hi = rp[row + 1];
      for (int64_t k = lo + sub; k < hi; k += L) s += (acc_t)rw_val(val, k) * (acc_t)x[col[k]];
    }
#pragma unroll
    for (int d = L / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, kWave);
    if (row < m && sub == 0) y[row] = (x_t)s;
  }
}

template <int DT>
int launch_rw(int lanes, const int32_t *rp, const int32_t *col, const void *val, const void *x, void *y, int64_t m,
              hipStream_t s) {
  int cus = 0, dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) { g_rw_hip = e; return SSS_ERR_HIP; }
  const int64_t rows_per_block = kThreads / lanes;
  // enough workgroups to fill the device several times over, grid-striding beyond
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((m + rows_per_block - 1) / rows_per_block,
                                                                (int64_t)cus * 16));
  const dim3 g((unsigned)blocks), b(kThreads);
  switch (lanes) {
    case 1: hipLaunchKernelGGL((sss_rowwise<DT, 1>), g, b, 0, s, rp, col, val, x, y, m); break;
    case 2: hipLaunchKernelGGL((sss_rowwise<DT, 2>), g, b, 0, s, rp, col, val, x, y, m); break;
    case 4: hipLaunchKernelGGL((sss_rowwise<DT, 4>), g, b, 0, s, rp, col, val, x, y, m); break;
    case 8: hipLaunchKernelGGL((sss_rowwise<DT, 8>), g, b, 0, s, rp, col, val, x, y, m); break;
    case 16: hipLaunchKernelGGL((sss_rowwise<DT, 16>), g, b, 0, s, rp, col, val, x, y, m); break;
    case 32: hipLaunchKernelGGL((sss_rowwise<DT, 32>), g, b, 0, s, rp, col, val, x, y, m); break;
    case 64: hipLaunchKernelGGL((sss_rowwise<DT, 64>), g, b, 0, s, rp, col, val, x, y, m); break;
    default: return SSS_ERR_UNSUPPORTED;
  }
  e = hipGetLastError();
  if (e != hipSuccess) { g_rw_hip = e; return SSS_ERR_HIP; }
  return SSS_OK;
}

}  // namespace

extern "C" {

int sss_csr_rowwise(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col, const void *val,
                    const void *x, void *y, sss_dtype dt, int lanes_per_row, void *stream) {
  if (m < 0 || n < 0 || nnz < 0 || m > SSS_MAX_INDEX || n > SSS_MAX_INDEX || nnz > SSS_MAX_INDEX)
    return SSS_ERR_INVALID_VALUE;
  if (!(lanes_per_row >= 1 && lanes_per_row <= kWave && (lanes_per_row & (lanes_per_row - 1)) == 0))
    return SSS_ERR_UNSUPPORTED;
  if (m == 0) return SSS_OK;
  if (!row_ptr || !y || (nnz > 0 && (!col || !val || !x))) return SSS_ERR_INVALID_VALUE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (dt) {
    case SSS_F64: return launch_rw<SSS_F64>(lanes_per_row, row_ptr, col, val, x, y, m, s);
    case SSS_F32: return launch_rw<SSS_F32>(lanes_per_row, row_ptr, col, val, x, y, m, s);
    case SSS_BF16: return launch_rw<SSS_BF16>(lanes_per_row, row_ptr, col, val, x, y, m, s);
    default: return SSS_ERR_UNSUPPORTED;
  }
}

const char *sss_rowwise_last_hip_error(void) { return hipGetErrorString(g_rw_hip); }

}  // extern "C"
