// Measurement aid, not part of the method: the device's rate of random
// gathers of x, independent of the method's tiling.
//
// Stage 1 of the speculative segmented sum reads a CSR matrix once as it is:
// col and val stream, and x is gathered at the columns (Section 2.1's
// products).  When the columns are spread over an x larger than an XCD's L2,
// those gathers, not the streaming, set the time (Section 4.4 measures
// bandwidth utilisation the same way).  This kernel measures how fast the
// device can serve such gathers at all, with none of stage 1's choices: every
// lane takes one nonzero per iteration of a grid-stride loop (k = thread +
// i * threads, so col and val are read coalesced), issues U gathers before it
// uses any, and the occupancy is set by reserving LDS.  Four ways to issue a
// gather are compared:
//   mode 0: plain vector loads;
//   mode 1: non-temporal vector loads (nt);
//   mode 2: direct-to-LDS loads (global_load_lds_dword): a gather in flight
//           holds no VGPR; each wave reads its lanes' values back from LDS;
//   mode 3: buffer loads at device scope (sc1), which the CU's L1 does not keep.
// Each thread writes one sum, so no load can be dropped.  Optionally the same
// kernel also moves the row part of a CSR SpMV's bytes, which the gathers do
// not: it reads row_ptr (m + 1 entries) and writes one value per row of y,
// both coalesced in a grid-stride loop interleaved with the gathers, so that
// a matrix with short rows is measured against every byte the product itself
// must move.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sss.h"

namespace {

constexpr int kProbeThreads = 256;  // 4 wavefronts per workgroup
constexpr int kWaveP = 64;
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr int kRowsInFlight = 4;  // row_ptr loads per thread before its y stores (8 cost the U = 16 instance two waves per SIMD)

thread_local hipError_t g_probe_hip = hipSuccess;

template <typename XT> struct Words { static constexpr int n = sizeof(XT) / 4; };

template <typename XT, int MODE>
__device__ __forceinline__ XT gather(const XT *__restrict__ x, __amdgpu_buffer_rsrc_t rsrc, int c) {
  if constexpr (MODE == 1) {
    return __builtin_nontemporal_load(x + c);
  } else if constexpr (MODE == 3) {
    if constexpr (sizeof(XT) == 8)
      return __builtin_bit_cast(XT, __builtin_amdgcn_raw_buffer_load_b64(rsrc, c * 8, 0, 16));
    else
      return __builtin_bit_cast(XT, __builtin_amdgcn_raw_buffer_load_b32(rsrc, c * 4, 0, 16));
  } else {
    return x[c];
  }
}

// U gathers of this lane, iterations k, k + stride, ..., k + (U-1) stride
// (all < nnz), summed (times val when WITH_VAL).
template <typename XT, int U, int MODE, bool WITH_VAL>
__device__ __forceinline__ XT probe_group(const int32_t *__restrict__ col, const XT *__restrict__ val,
                                          const XT *__restrict__ x, __amdgpu_buffer_rsrc_t rsrc, int64_t k,
                                          int64_t stride, uint32_t *lds_wave, int lane) {
  int c[U];
  XT a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    c[u] = col[k + u * stride];
    if constexpr (WITH_VAL) a[u] = val[k + u * stride];
  }
  // the three phases (index and value loads, gathers, use) stay apart, so
  // that all U gathers are in flight before the first is used
  __builtin_amdgcn_sched_barrier(0);
  XT acc = 0;
  if constexpr (MODE == 2) {
    // slot u, word w of this wave's LDS: 64 lanes x 4 bytes each
    constexpr int NW = Words<XT>::n;
    const uint32_t *xw = reinterpret_cast<const uint32_t *>(x);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int w = 0; w < NW; ++w)
        __builtin_amdgcn_global_load_lds(xw + (int64_t)c[u] * NW + w, lds_wave + (u * NW + w) * kWaveP, 4, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);  // the LDS writes of this wave's loads have landed
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      XT v;
      if constexpr (NW == 2) {
        const uint64_t lo = lds_wave[(u * 2) * kWaveP + lane], hi = lds_wave[(u * 2 + 1) * kWaveP + lane];
        v = __builtin_bit_cast(XT, lo | (hi << 32));
      } else {
        v = __builtin_bit_cast(XT, lds_wave[u * kWaveP + lane]);
      }
      acc += WITH_VAL ? a[u] * v : v;
    }
    __builtin_amdgcn_wave_barrier();  // every lane has read its slots before they are reused
  } else {
    XT v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = gather<XT, MODE>(x, rsrc, c[u]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += WITH_VAL ? a[u] * v[u] : v[u];
  }
  return acc;
}

// CHUNKED = false: one grid-stride loop over all nonzeros (the whole grid
// sweeps the matrix as one front).  CHUNKED = true: every wavefront sweeps
// its own contiguous chunk of the nonzeros, 64 at a time (lane + 64 i), as a
// thread-bunch of the method does.  ROWS: also the row part (its registers
// would otherwise lower the occupancy of the instances without it).
template <typename XT, int U, int MODE, bool WITH_VAL, bool CHUNKED, bool ROWS>
__global__ __launch_bounds__(kProbeThreads) void sss_gather_probe_kernel(const int32_t *__restrict__ col,
                                                                         const XT *__restrict__ val,
                                                                         const XT *__restrict__ x, int64_t nnz,
                                                                         int64_t n, XT *__restrict__ out,
                                                                         const int32_t *__restrict__ rp, int64_t m,
                                                                         XT *__restrict__ y, int rows_after) {
  extern __shared__ uint32_t lds_probe[];
  const int lane = threadIdx.x & (kWaveP - 1);
  uint32_t *lds_wave = lds_probe + (threadIdx.x / kWaveP) * (U * Words<XT>::n * kWaveP);
  const __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<XT *>(x), 0, (int)(n * (int64_t)sizeof(XT)), 0x00020000);
  const int64_t threads = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = threads, begin = t - lane, end = nnz;
  if constexpr (CHUNKED) {
    const int64_t waves = threads / kWaveP;
    const int64_t chunk = ((nnz + waves - 1) / waves + kWaveP - 1) / kWaveP * kWaveP;
    stride = kWaveP;
    begin = (t / kWaveP) * chunk;
    end = begin + chunk < nnz ? begin + chunk : nnz;
  }
  XT acc = 0;
  int64_t k = begin + lane;
  // the row part (row_ptr read once, y written once, over the whole grid) in
  // batches of kRowsInFlight rows per thread, loads before stores; the
  // batches are spread over the nonzero groups, so that row and gather
  // traffic share the run as they do in a product, or (rows_after) all follow
  // the gathers
  const int64_t rows_step = (int64_t)kRowsInFlight * threads;
  const int64_t n_rb = ROWS ? (m + rows_step) / rows_step : 0;  // ceil((m + 1) / rows_step)
  const bool spread = n_rb > 0 && !rows_after;
  const int64_t n_groups = (end - begin + (int64_t)U * stride - 1) / ((int64_t)U * stride);
  int64_t rb = 0, g = 0;
  auto row_batches = [&](int64_t upto) {
    if constexpr (!ROWS) return;
    for (; rb < upto; ++rb) {
      const int64_t r0 = t + rb * rows_step;
      int32_t v[kRowsInFlight];
#pragma unroll
      for (int u = 0; u < kRowsInFlight; ++u) {
        const int64_t r = r0 + u * threads;
        v[u] = r <= m ? rp[r] : 0;
      }
#pragma unroll
      for (int u = 0; u < kRowsInFlight; ++u) {
        const int64_t r = r0 + u * threads;
        if (r < m) y[r] = (XT)v[u];
        else if (r == m) acc += (XT)v[u];
      }
    }
  };
  // full groups: the group's last iteration is inside for every lane of the
  // wave when it is for the wave's last lane, so the LDS path stays
  // wave-uniform
  for (int64_t wave_last = begin + (kWaveP - 1); wave_last + (int64_t)(U - 1) * stride < end;
       wave_last += (int64_t)U * stride, k += (int64_t)U * stride) {
    acc += probe_group<XT, U, MODE, WITH_VAL>(col, val, x, rsrc, k, stride, lds_wave, lane);
    ++g;
    if (ROWS && spread) row_batches((g * n_rb + n_groups - 1) / n_groups);
  }
  for (; k < end; k += stride) {
    const XT v = x[col[k]];
    acc += WITH_VAL ? val[k] * v : v;
  }
  row_batches(n_rb);
  out[t] = acc;
}

template <typename XT, int MODE, bool WITH_VAL, bool CHUNKED, bool ROWS>
const void *pick_u(int U) {
  switch (U) {
    case 1: return reinterpret_cast<const void *>(sss_gather_probe_kernel<XT, 1, MODE, WITH_VAL, CHUNKED, ROWS>);
    case 2: return reinterpret_cast<const void *>(sss_gather_probe_kernel<XT, 2, MODE, WITH_VAL, CHUNKED, ROWS>);
    case 4: return reinterpret_cast<const void *>(sss_gather_probe_kernel<XT, 4, MODE, WITH_VAL, CHUNKED, ROWS>);
    case 8: return reinterpret_cast<const void *>(sss_gather_probe_kernel<XT, 8, MODE, WITH_VAL, CHUNKED, ROWS>);
    case 16: return reinterpret_cast<const void *>(sss_gather_probe_kernel<XT, 16, MODE, WITH_VAL, CHUNKED, ROWS>);
    default: return nullptr;
  }
}

template <typename XT, bool WITH_VAL, bool CHUNKED, bool ROWS>
const void *pick_mode(int mode, int U) {
  switch (mode) {
    case 0: return pick_u<XT, 0, WITH_VAL, CHUNKED, ROWS>(U);
    case 1: return pick_u<XT, 1, WITH_VAL, CHUNKED, ROWS>(U);
    case 2: return pick_u<XT, 2, WITH_VAL, CHUNKED, ROWS>(U);
    case 3: return pick_u<XT, 3, WITH_VAL, CHUNKED, ROWS>(U);
    default: return nullptr;
  }
}

template <typename XT, bool ROWS>
const void *pick_kernel(int mode, int U, bool with_val, bool chunked) {
  if (with_val)
    return chunked ? pick_mode<XT, true, true, ROWS>(mode, U) : pick_mode<XT, true, false, ROWS>(mode, U);
  return chunked ? pick_mode<XT, false, true, ROWS>(mode, U) : pick_mode<XT, false, false, ROWS>(mode, U);
}

}  // namespace

extern "C" {

int sss_gather_probe_rows(const int32_t *col, const void *val, const void *x, int64_t nnz, int64_t n, sss_dtype dt,
                          int mode, int unroll, int waves_per_simd, int with_val, void *out, int64_t out_len,
                          int64_t *threads, int *resident_per_cu, const int32_t *row_ptr, int64_t m, void *y,
                          void *stream) {
  if (nnz < 0 || n < 1 || nnz > SSS_MAX_INDEX || n > SSS_MAX_INDEX / 8 || !col || !x || !out || !threads ||
      (with_val && !val) || (row_ptr && (m < 0 || m > SSS_MAX_INDEX || (m > 0 && !y))))
    return SSS_ERR_INVALID_VALUE;
  if (!row_ptr) { m = 0; y = nullptr; }
  if (dt != SSS_F64 && dt != SSS_F32) return SSS_ERR_UNSUPPORTED;
  if (!(waves_per_simd == 1 || waves_per_simd == 2 || waves_per_simd == 4 || waves_per_simd == 8))
    return SSS_ERR_INVALID_VALUE;
  const bool chunked = (mode & 4) != 0;
  int rows_after = (mode & 8) != 0;
  mode &= 3;
  const bool rows = row_ptr != nullptr;
  const void *k = dt == SSS_F64 ? (rows ? pick_kernel<double, true>(mode, unroll, with_val != 0, chunked)
                                        : pick_kernel<double, false>(mode, unroll, with_val != 0, chunked))
                                : (rows ? pick_kernel<float, true>(mode, unroll, with_val != 0, chunked)
                                        : pick_kernel<float, false>(mode, unroll, with_val != 0, chunked));
  if (!k) return SSS_ERR_UNSUPPORTED;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) { g_probe_hip = e; return SSS_ERR_HIP; }
  // a workgroup is one wavefront per SIMD: waves_per_simd workgroups per CU,
  // held there by each reserving 1/waves_per_simd of the CU's LDS (fewer if
  // the kernel's registers allow fewer), so every workgroup is resident at
  // once and the grid-stride loop has no second round
  const size_t words = (size_t)unroll * (dt == SSS_F64 ? 2 : 1) * kWaveP * (kProbeThreads / kWaveP);
  const size_t need = mode == 2 ? words * 4 : 0;
  const size_t lds = (kLdsPerCu / waves_per_simd) & ~(size_t)1023;
  if (need > lds) return SSS_ERR_UNSUPPORTED;
  e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int per_cu = 0;
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kProbeThreads, lds);
  if (e != hipSuccess) { g_probe_hip = e; return SSS_ERR_HIP; }
  if (per_cu < 1) return SSS_ERR_UNSUPPORTED;
  if (resident_per_cu) *resident_per_cu = per_cu;
  const int64_t blocks = (int64_t)cus * per_cu;
  *threads = blocks * kProbeThreads;
  if (out_len < *threads) return SSS_ERR_INVALID_VALUE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void *args[] = {&col, &val, &x, &nnz, &n, &out, &row_ptr, &m, &y, &rows_after};
  e = hipLaunchKernel(k, dim3((unsigned)blocks), dim3(kProbeThreads), args, lds, s);
  if (e != hipSuccess) { g_probe_hip = e; return SSS_ERR_HIP; }
  return SSS_OK;
}

int sss_gather_probe(const int32_t *col, const void *val, const void *x, int64_t nnz, int64_t n, sss_dtype dt,
                     int mode, int unroll, int waves_per_simd, int with_val, void *out, int64_t out_len,
                     int64_t *threads, int *resident_per_cu, void *stream) {
  return sss_gather_probe_rows(col, val, x, nnz, n, dt, mode, unroll, waves_per_simd, with_val, out, out_len, threads,
                               resident_per_cu, nullptr, 0, nullptr, stream);
}

const char *sss_probe_last_hip_error(void) { return hipGetErrorString(g_probe_hip); }

}  // extern "C"
