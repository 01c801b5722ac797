// Speculative segmented sum CSR SpMV for gfx950 (MI355X), y = A x.
//
// Stage 1 (Section 3.2, the appendix algorithm's first-stage function): one
// 64-lane wavefront per thread-bunch of S tiles, each tile W*64 nonzeros
// (Section 3.1).  Per bunch:
//   * the bunch's first row r0 = rightmost row with row_ptr[r] <= b0, by a
//     wave-parallel 64-ary search (each round narrows the range 64x with one
//     load per lane and a ballot), or read from the plan when the plan ran
//     that search once for all calls (bound rows);
//   * one pass over the bunch's rows in 64-row chunks builds the segment
//     descriptor of all S tiles as a bit mask in LDS (head at row_ptr[r] - b0
//     for each non-empty row), finds every tile's start row (the rightmost
//     match of each tile boundary, counted by ballots) and detects the dirty
//     tiles (an empty row among rows start..stop-1 of the tile);
//   * per tile: coalesced vector loads of col/val in a grouped order (lane
//     j loads G consecutive entries of each row of 64*G; 16 bytes of values
//     per load), gathers of x in the same order, the products moved through
//     LDS to lane j's entries [jW, jW+W), an exclusive scan of head counts giving each
//     partial sum its compact rank q, one pass over the lane's products that
//     stores every segment closed inside the lane, a 64-lane segmented scan
//     of the lanes' open segments (DPP) that completes the segments crossing
//     lanes, and the store of partial q to y[start + q].
//     The bunch's first segment goes to the synchronizer instead; a tile that
//     ends inside row `stop` hands its last partial to the next tile through
//     the transmitter.  Dirty tiles are recorded, as <start, stop, tile>, in
//     the bunch's own speculator slots, with a per-bunch dirty mask.
// Stage 2 (Section 3.2, checking prediction; the paper runs it on a CPU core)
// is one device kernel with three independent parts: the synchronizer carries
// (one thread per run of bunches sharing a first row; the wavefront for long
// runs), the re-arrangement of each dirty tile's partial sums to its non-empty
// rows (one wavefront per thread-bunch), and zeroing the leading empty rows no
// tile covers.
//
// Differences from the paper's listing, on purpose:
//  * a dirty tile that ends inside row `stop` also passes its last partial on
//    through the transmitter and writes it at y[stop] (its true row), where
//    the listing clears the transmitter and leaves that partial to the
//    re-arrangement.  The result is the same sum; the gain is that the
//    re-arrangement then only touches rows strictly inside dirty tiles, so all
//    three parts of stage 2 are disjoint and run concurrently in one launch,
//    with no ordering between them.
//  * the speculator is packed per thread-bunch (S slots each, plus a dirty
//    mask) instead of through one global atomic counter.  On a multi-die GPU a
//    device-wide counter needs either a cross-die atomic per dirty tile and a
//    grid-wide "last block" handshake to reset it between calls, or an extra
//    launch; per-bunch slots need neither, and stage 2's wavefront for a bunch
//    finds that bunch's dirty tiles directly.
//
// Precision: F64 sums in double.  F32/BF16 multiply in float and sum segments
// with TwoSum-compensated float pairs; each partial is formed in double, the
// transmitter, the synchronizer and the stage-2 carry sums are double.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <climits>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "sss.h"

namespace {

constexpr int kWave = 64;
constexpr int kShortRun = 16;  // stage-2 carry runs up to this many bunches: one thread

thread_local hipError_t g_last_hip = hipSuccess;

#define SSS_HIP(call)                         \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) {                   \
      g_last_hip = e_;                        \
      return SSS_ERR_HIP;                     \
    }                                         \
  } while (0)

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

#ifndef SSS_NT_LOADS
#define SSS_NT_LOADS 0
#endif
#ifndef SSS_NT_STORES
#define SSS_NT_STORES 0
#endif
#ifndef SSS_WAVES_PER_EU
#define SSS_WAVES_PER_EU 0
#endif

// streaming loads of the matrix arrays (plain loads stream faster than
// non-temporal ones on gfx950 for this pattern)
template <typename T>
__device__ __forceinline__ T stream_load(const T *p) {
  if constexpr (SSS_NT_LOADS) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T>
__device__ __forceinline__ void y_store(T v, T *p) {
  if constexpr (SSS_NT_STORES) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ---------------------------------------------------------------- value types

template <int DT> struct VT;
template <> struct VT<SSS_F64> { using val_t = double;   using x_t = double; using y_t = double; using prod_t = double; };
template <> struct VT<SSS_F32> { using val_t = float;    using x_t = float;  using y_t = float;  using prod_t = float; };
template <> struct VT<SSS_BF16>{ using val_t = uint16_t; using x_t = float;  using y_t = float;  using prod_t = float; };

__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) {
  return __uint_as_float(bits16 << 16);
}

// Accumulators.  F64: one double.  F32/BF16: an unevaluated float pair
// (hi, lo) kept by TwoSum (Knuth), i.e. compensated summation.
struct AccD {
  double s;
  __device__ __forceinline__ void zero() { s = 0.0; }
  __device__ __forceinline__ void add(double v) { s += v; }
  // this := earlier (+) this
  __device__ __forceinline__ void prepend(const AccD &earlier) { s = earlier.s + s; }
  __device__ __forceinline__ double value() const { return s; }
  __device__ __forceinline__ AccD shfl_up(unsigned d) const { AccD r; r.s = __shfl_up(s, d, kWave); return r; }
};

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  const float z = s - a;
  e = (a - (s - z)) + (b - z);
}

struct AccC {
  float hi, lo;
  __device__ __forceinline__ void zero() { hi = 0.f; lo = 0.f; }
  __device__ __forceinline__ void add(float v) {
    float s, e;
    two_sum(hi, v, s, e);
    hi = s;
    lo += e;
  }
  // this := earlier (+) this, as a float pair
  __device__ __forceinline__ void prepend(const AccC &earlier) {
    float s, e;
    two_sum(earlier.hi, hi, s, e);
    e += earlier.lo + lo;
    hi = s + e;  // renormalise (fast two-sum; |s| >= |e| up to rounding)
    lo = e - (hi - s);
  }
  __device__ __forceinline__ double value() const { return (double)hi + (double)lo; }
  __device__ __forceinline__ AccC shfl_up(unsigned d) const {
    AccC r;
    r.hi = __shfl_up(hi, d, kWave);
    r.lo = __shfl_up(lo, d, kWave);
    return r;
  }
};

template <int DT> struct AccSel { using type = AccC; };
template <> struct AccSel<SSS_F64> { using type = AccD; };
template <int DT> using Acc = typename AccSel<DT>::type;

// ---------------------------------------------------------------- loads

__device__ __forceinline__ double scalar_val(const double *v, int k) { return v[k]; }
__device__ __forceinline__ float scalar_val(const float *v, int k) { return v[k]; }
__device__ __forceinline__ float scalar_val(const uint16_t *v, int k) { return bf16_to_f32(v[k]); }

// Integer minimum (HIP's min for 64-bit integers goes through double).
__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

// ---------------------------------------------------------------- search

// Largest r in [0, m] with rp[r] <= b (rp non-decreasing, rp[0] <= b).
// Wave-parallel 64-ary search: each round the 64 lanes probe 64 evenly spaced
// points of (lo, hi]; the predicate rp[p] <= b holds for a prefix of lanes, so
// its ballot's popcount picks the sub-interval.
template <typename T, typename I>
__device__ __forceinline__ I wave_rightmost(const T *__restrict__ rp, I m, T b, int lane) {
  I lo = 0, hi = m;
  while (hi - lo >= kWave) {
    const int64_t span = (int64_t)(hi - lo);
    const I p = lo + (I)(((int64_t)(lane + 1) * span) / kWave);
    const uint64_t bal = __ballot(rp[p] <= b);
    const int c = __popcll(bal);
    const I newlo = c > 0 ? lo + (I)(((int64_t)c * span) / kWave) : lo;
    const I newhi = c < kWave ? lo + (I)(((int64_t)(c + 1) * span) / kWave) - 1 : hi;
    lo = newlo;
    hi = newhi;
  }
  const I p = lo + lane;
  const bool pred = (p <= hi) && (rp[p <= hi ? p : hi] <= b);
  return lo + __popcll(__ballot(pred)) - 1;
}

// ---------------------------------------------------------------- wave scans

// 64-lane scans with DPP: Hillis-Steele shifts by 1, 2, 4, 8 inside each
// 16-lane row, then row broadcasts of lane 15 (into rows 1 and 3) and lane 31
// (into rows 2 and 3).  Lanes whose source is out of range read 0, the
// identity of both scans below.
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143, kWaveShr1 = 0x138, kWaveShl1 = 0x130;

// lane l reads lane l + 1; the last lane keeps `last`
__device__ __forceinline__ int wave_next(int v, int last) {
  return __builtin_amdgcn_update_dpp(last, v, kWaveShl1, 0xf, 0xf, false);
}
// lane l reads lane l - 1; lane 0 keeps `first`
__device__ __forceinline__ int wave_prev(int v, int first) {
  return __builtin_amdgcn_update_dpp(first, v, kWaveShr1, 0xf, 0xf, false);
}
// v of lane `l`, for a lane index the same in every lane
__device__ __forceinline__ int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
// a 64-bit value the same in every lane, in scalar registers
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// *p for an address the same in every lane, of data no kernel of the launch
// writes (plan arrays written before it): read through the scalar unit into
// scalar registers instead of once per lane into vector registers
template <typename T>
__device__ __forceinline__ T uniform_load(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
  typedef const __attribute__((address_space(4))) uint32_t cword;
  uint32_t w[sizeof(T) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = ((cword *)p)[i];
  T v;
  __builtin_memcpy(&v, w, sizeof(T));
  return v;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL, ROWS>(__float_as_int(v)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL, ROWS>((int)(unsigned long long)b);
  const int hi = dpp_i<CTRL, ROWS>((int)((unsigned long long)b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ AccD dpp_acc(const AccD &v) { AccD r; r.s = dpp_d<CTRL, ROWS>(v.s); return r; }
template <int CTRL, int ROWS>
__device__ __forceinline__ AccC dpp_acc(const AccC &v) {
  AccC r;
  r.hi = dpp_f<CTRL, ROWS>(v.hi);
  r.lo = dpp_f<CTRL, ROWS>(v.lo);
  return r;
}

// one step of the segmented scan: (v, f) := (v_src, f_src) (+) (v, f), where
// (a, fa) (+) (b, fb) = (fb ? b : a + b, fa | fb)
template <int CTRL, int ROWS, class A>
__device__ __forceinline__ void seg_step(A &v, int &f) {
  const A up = dpp_acc<CTRL, ROWS>(v);
  const int fu = dpp_i<CTRL, ROWS>(f);
  if (!f) v.prepend(up);
  f |= fu;
}

// inclusive segmented scan over the wave of (v, head flag)
template <class A>
__device__ __forceinline__ void wave_seg_scan(A &v, int &f) {
  seg_step<kRowShr1, 0xf>(v, f);
  seg_step<kRowShr2, 0xf>(v, f);
  seg_step<kRowShr4, 0xf>(v, f);
  seg_step<kRowShr8, 0xf>(v, f);
  seg_step<kRowBcast15, 0xa>(v, f);
  seg_step<kRowBcast31, 0xc>(v, f);
}

// inclusive integer scan over the wave
__device__ __forceinline__ int wave_iscan(int x) {
  x += dpp_i<kRowShr1, 0xf>(x);
  x += dpp_i<kRowShr2, 0xf>(x);
  x += dpp_i<kRowShr4, 0xf>(x);
  x += dpp_i<kRowShr8, 0xf>(x);
  x += dpp_i<kRowBcast15, 0xa>(x);
  x += dpp_i<kRowBcast31, 0xc>(x);
  return x;
}

// sum over the 64 lanes in a fixed tree (pairs 1 apart, 2 apart, ... 32
// apart); every lane returns the total
__device__ __forceinline__ double wave_sum_tree(double v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// ---------------------------------------------------------------- stage 1

// One matrix as the kernels see it: the caller's arrays, sizes, and the
// plan's auxiliary arrays for this matrix (already offset to it).
struct MatCtx {
  const int32_t *row_ptr;
  const int32_t *col;
  const void *val;
  const void *x;
  void *y;
  int32_t m;
  int32_t nnz;
  int32_t S;
  int32_t W;
  int64_t n_bunches;
  int64_t n_tiles;
  uint32_t *dirty_mask;  // per bunch: bit t set when its tile t is dirty
  int4 *speculator;      // per bunch, S slots: <start, stop, tile, 0> of its dirty tiles, packed
  int32_t *sync_idx;
  double *sync_val;
  double *tail_val;      // per bunch: its last partial, when the bunch ends inside a row that is not
                         // its first row and continues into the next bunch (written only then)
  const int32_t *bunch_row;  // per bunch: its first row, found at plan time (NULL: search); the top
                             // bit is set on the bunches listed in dirty_list
  const int32_t *dirty_list; // bound plans: the bunches whose tiles the plan found dirty (NULL: every
                             // bunch gets a stage-2 wavefront)
  int64_t n_fix;             // stage-2 re-arrangement wavefronts: entries of dirty_list, else n_bunches
  int32_t *stale;            // bound plans: set (and never cleared) when stage 1 finds a dirty tile in a
                             // bunch outside dirty_list (row_ptr rewritten in place since plan time)
  int32_t *dbg_start;    // debug plans only
  int32_t *dbg_dirty;
  uint32_t *dbg_heads;
};

// LDS words per wavefront: S tiles of descriptor bits, the dirty-tile bits
// (padded to 2 words), then W*T double slots for one tile's compact partials.
__host__ __device__ constexpr int stage1_lds_words(int W, int S) { return S * (W * kWave / 32) + 2 + 2 * W * kWave; }

// Grouped order of a tile's entries: the tile is W/G rows of 64*G entries,
// and lane j holds G consecutive entries of every row, so entry (r, g) of
// lane j (array index r*G + g) is tile offset r*64*G + j*G + g.  G entries
// of the value type make 16 bytes (G = W when that is fewer), so every load
// instruction of the wavefront reads one contiguous 1-KiB stretch of val,
// and the x gathers of one instruction fall on 64*G consecutive nonzeros.
template <int DT> constexpr int group_of() { return DT == SSS_F64 ? 2 : (DT == SSS_F32 ? 4 : 8); }
template <int DT, int W> constexpr int group_w() { return group_of<DT>() < W ? group_of<DT>() : W; }

template <int G>
__device__ __forceinline__ void load_cols_g(const int32_t *__restrict__ p, int *c) {
  if constexpr (G == 2) {
    const v2u v = stream_load(reinterpret_cast<const v2u *>(p));
    c[0] = (int)v.x; c[1] = (int)v.y;
  } else {
#pragma unroll
    for (int i = 0; i < G / 4; ++i) {
      const v4i v = stream_load(reinterpret_cast<const v4i *>(p) + i);
      c[4 * i] = v.x; c[4 * i + 1] = v.y; c[4 * i + 2] = v.z; c[4 * i + 3] = v.w;
    }
  }
}

template <int G>
__device__ __forceinline__ void load_vals_g(const double *__restrict__ p, double *a) {
  static_assert(G % 2 == 0, "double groups are pairs");
#pragma unroll
  for (int i = 0; i < G / 2; ++i) {
    const v2d v = stream_load(reinterpret_cast<const v2d *>(p) + i);
    a[2 * i] = v.x; a[2 * i + 1] = v.y;
  }
}
template <int G>
__device__ __forceinline__ void load_vals_g(const float *__restrict__ p, float *a) {
  static_assert(G % 4 == 0, "float groups are quadruples");
#pragma unroll
  for (int i = 0; i < G / 4; ++i) {
    const v4f v = stream_load(reinterpret_cast<const v4f *>(p) + i);
    a[4 * i] = v.x; a[4 * i + 1] = v.y; a[4 * i + 2] = v.z; a[4 * i + 3] = v.w;
  }
}
template <int G>
__device__ __forceinline__ void load_vals_g(const uint16_t *__restrict__ p, float *a) {
  if constexpr (G == 8) {
    const v4u v = stream_load(reinterpret_cast<const v4u *>(p));
    const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) { a[2 * j] = bf16_to_f32(w[j] & 0xffffu); a[2 * j + 1] = bf16_to_f32(w[j] >> 16); }
  } else {
    static_assert(G == 4, "bfloat16 groups are 4 or 8");
    const v2u v = stream_load(reinterpret_cast<const v2u *>(p));
    a[0] = bf16_to_f32(v.x & 0xffffu); a[1] = bf16_to_f32(v.x >> 16);
    a[2] = bf16_to_f32(v.y & 0xffffu); a[3] = bf16_to_f32(v.y >> 16);
  }
}

// col/val of one tile in the grouped order; entries past nnz read as column 0
// with value 0.
template <int DT, int W, typename val_t, typename prod_t>
__device__ __forceinline__ void load_tile_g(const int32_t *__restrict__ col, const val_t *__restrict__ val, int b,
                                            int nnz, int lane, int (&c)[W], prod_t (&av)[W]) {
  constexpr int G = group_w<DT, W>();
  constexpr int R = W / G;
  if (b + W * kWave <= nnz) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k0 = b + r * kWave * G + lane * G;
      load_cols_g<G>(col + k0, &c[r * G]);
      load_vals_g<G>(val + k0, &av[r * G]);
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int k = b + r * kWave * G + lane * G + g;
        const bool in = k < nnz;
        c[r * G + g] = in ? col[k] : 0;
        av[r * G + g] = in ? (prod_t)scalar_val(val, k) : (prod_t)0;
      }
  }
}

// The products leave the grouped order through LDS: each lane writes its G
// products of every row as 16-byte chunks, then reads back the W products
// of tile offsets lane*W .. lane*W+W-1 (the order the segmented sum walks).
// 16-byte chunk c is stored at chunk c ^ ((c >> 4) & (K - 1)), K = the chunks
// one lane reads: the 16 lanes of a read then touch 16 different chunk
// columns of a 256-byte LDS row, as do the lanes of a write.
template <typename P, int W>
__device__ __forceinline__ int tr_chunk(int c) {
  constexpr int K = (W * (int)sizeof(P)) / 16 > 0 ? (W * (int)sizeof(P)) / 16 : 1;
  return c ^ ((c >> 4) & (K - 1));
}

template <int DT, int W, typename P>
__device__ __forceinline__ void products_out(const P (&av)[W], const P (&xv)[W], P *buf, int lane, P (&pr)[W]) {
  constexpr int G = group_w<DT, W>();
  constexpr int R = W / G;
  constexpr int CH = 16 / (int)sizeof(P);  // products per 16-byte chunk
  static_assert(W % CH == 0, "a lane's products fill whole chunks");
  if constexpr (G == W) {
    // one row per tile: the grouped order is the lane order already
#pragma unroll
    for (int i = 0; i < W; ++i) pr[i] = av[i] * xv[i];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < G / CH; ++t) {
        const int c = (r * kWave * G + lane * G) / CH + t;
        P *dst = buf + tr_chunk<P, W>(c) * CH;
#pragma unroll
        for (int e = 0; e < CH; ++e) dst[e] = av[r * G + t * CH + e] * xv[r * G + t * CH + e];
      }
  }
}

template <int DT, int W, typename P>
__device__ __forceinline__ void products_in(const P *buf, int lane, P (&pr)[W]) {
  constexpr int CH = 16 / (int)sizeof(P);
  if constexpr (group_w<DT, W>() != W) {
    // one wavefront owns buf and its LDS operations run in order; the
    // fence keeps the compiler from moving a read above another lane's write
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < W / CH; ++k) {
      const P *src = buf + tr_chunk<P, W>((lane * W) / CH + k) * CH;
#pragma unroll
      for (int e = 0; e < CH; ++e) pr[k * CH + e] = src[e];
    }
  }
}

template <int DT, int W, bool DEBUG>
__device__ __forceinline__ void stage1_bunch(const MatCtx &a, const int64_t tb, uint32_t *lds_wave, const int lane,
                                             const int32_t brow) {
  using val_t = typename VT<DT>::val_t;
  using x_t = typename VT<DT>::x_t;
  using y_t = typename VT<DT>::y_t;
  using prod_t = typename VT<DT>::prod_t;
  constexpr int WT = W * kWave;
  constexpr int WPT = WT / 32;  // descriptor words per tile
  constexpr uint32_t LOW = (W >= 32) ? 0xffffffffu : ((1u << W) - 1u);

  const int32_t *__restrict__ rp = a.row_ptr;
  const int32_t *__restrict__ col = a.col;
  const val_t *__restrict__ val = static_cast<const val_t *>(a.val);
  const x_t *__restrict__ x = static_cast<const x_t *>(a.x);
  y_t *__restrict__ y = static_cast<y_t *>(a.y);
  const int m = a.m, nnz = a.nnz, S = a.S;
  uint32_t *mask = lds_wave;
  uint32_t *dflag = mask + S * WPT;
  double *part = reinterpret_cast<double *>(mask + S * WPT + 2);

  const int64_t SWT = (int64_t)S * WT;
  const int b0 = (int)(tb * SWT);  // < nnz
  const int bS = (int)imin64(tb * SWT + SWT, nnz);

  // ---- tile 0's col/val do not depend on the row structure: issue first
  int cc[W];
  prod_t av[W];
  load_tile_g<DT, W>(col, val, b0, nnz, lane, cc, av);

  // ---- tile boundary search (rightmost match) for the bunch's first row,
  // unless the plan found it once for all calls; such a row is checked in the
  // row pass below
  // brow: -1 = search for the first row; else the first row found at plan
  // time, top bit set when the plan listed this bunch as dirty (decoded
  // here, after tile 0's loads are issued, so nothing waits for it earlier)
  const bool known = brow != -1;
  const bool listed = brow < 0;
  int r0 = known ? (brow & 0x7fffffff) : wave_rightmost(rp, m, b0, lane);
  bool verify = known;

  // ---- x gathers of tile 0: they need only the columns, so they go out
  // before the row pass and travel with its loads
  prod_t xv[W];
#pragma unroll
  for (int i = 0; i < W; ++i) xv[i] = (prod_t)x[cc[i]];

  // ---- descriptor, tile start rows, dirty tiles: one pass over the rows
  for (int i = lane; i < S * WPT; i += kWave) mask[i] = 0u;
  if (lane == 0) *dflag = 0u;
  __builtin_amdgcn_wave_barrier();

  const int my_b = (int)imin64(tb * SWT + (int64_t)min(lane, S) * WT, nnz);
  int my_count = 0;  // lane t <= S: rows r >= r0 with rp[r] <= b_t
  int my_rp = 0;     // lane t <= S: rp of the last such row (the tile's start row)
  for (int rbase = __builtin_amdgcn_readfirstlane(r0);; rbase += kWave) {
    const int r = rbase + lane;
    const int p = (r <= m) ? rp[r] : INT_MAX;
    // q = rp[r + 1]: the next lane's p, and one uniform load for the last lane
    const int q = wave_next(p, (rbase + kWave - 1 < m) ? rp[rbase + kWave] : INT_MAX);
    if (verify) {
      // a row found at plan time is the rightmost match of b0 exactly when
      // rp[r0] <= b0 < rp[r0 + 1]; if row_ptr no longer says so, search
      // (the pass has accumulated nothing yet)
      verify = false;
      const int p0 = lane_value(p, 0), q0 = lane_value(q, 0);
      if (!(p0 <= b0 && b0 < q0)) {
        r0 = __builtin_amdgcn_readfirstlane(wave_rightmost(rp, m, b0, lane));
        rbase = r0 - kWave;
        continue;
      }
    }
    if (r < m && q > p && p >= b0 && p < bS) {
      const int off = p - b0;
      atomicOr(&mask[off >> 5], 1u << (off & 31));
    }
    // an empty row at position p lies in rows start..stop-1 of the tile t
    // with b_t < p <= b_{t+1}
    if (r < m && q == p && p > b0 && p <= bS) atomicOr(dflag, 1u << ((p - b0 - 1) / WT));
    for (int t = 0; t <= S; ++t) {
      // rows with rp <= b_t are a prefix of the chunk; the last of them
      // (so far) is the start row of tile t
      const int bt = lane_value(my_b, t);
      const int c = __popcll(__ballot(p <= bt));
      const int p_last_in = lane_value(p, c > 0 ? c - 1 : 0);
      if (lane == t) {
        my_count += c;
        if (c > 0) my_rp = p_last_in;
      }
    }
    const int p_last = lane_value(p, kWave - 1);
    if (!(p_last <= bS && rbase + (kWave - 1) < m)) break;
  }
  __builtin_amdgcn_wave_barrier();
  const uint32_t dirty_bits = *dflag;
  const int my_start = (lane <= S) ? r0 + my_count - 1 : 0;

  double transmitter = 0.0;
  double sync_v = 0.0;
  for (int t = 0; t < S; ++t) {
    const int64_t b64 = tb * SWT + (int64_t)t * WT;
    if (b64 >= nnz) break;
    const int b = (int)b64;
    const int e = (int)imin64(b64 + WT, nnz);
    const int start = lane_value(my_start, t);
    const int stop = lane_value(my_start, t + 1);
    const int rp_stop = lane_value(my_rp, t + 1);
    const bool ends_mid = (stop < m) && (rp_stop < e);
    const bool dirty = (dirty_bits >> t) & 1u;
    const int64_t tile = tb * S + t;
    const bool has_next = (t + 1 < S) && (b64 + WT < nnz);

    // ---- prefetch the next tile's col/val; products of this tile
    int cn[W];
    prod_t an[W];
    if (has_next) load_tile_g<DT, W>(col, val, b + WT, nnz, lane, cn, an);
    // ---- this lane's W descriptor bits; the tile's first bit is forced
    uint32_t hb = (mask[t * WPT + ((lane * W) >> 5)] >> ((lane * W) & 31)) & LOW;
    const bool bit0 = __builtin_amdgcn_readlane((int)hb, 0) & 1;
    if (lane == 0) hb |= 1u;
    const double tx = bit0 ? 0.0 : transmitter;  // carry into a tile that starts mid-row
    if (DEBUG) {
      for (int w = lane; w < WPT; w += kWave) {
        uint32_t word = mask[t * WPT + w];
        if (w == 0) word |= 1u;
        a.dbg_heads[tile * WPT + w] = word;
      }
      if (lane == 0) {
        a.dbg_start[tile] = start;
        a.dbg_dirty[tile] = dirty ? 1 : 0;
      }
    }

    // ---- exclusive scan of head counts: the compact index of every partial
    // (integers only, so it does not wait for the products)
    const int c_heads = __popc(hb);
    const int incl = wave_iscan(c_heads);
    const int cnt = __builtin_amdgcn_readlane(incl, kWave - 1);
    const int rank0 = incl - c_heads;  // segments closed before this lane's first head

    // ---- one pass over the lane's products.  `pre` = the entries before the
    // lane's first head (they continue a segment opened in an earlier lane);
    // every later head closes a segment that lies wholly in this lane, whose
    // partial goes to its LDS slot at once; `run` = the entries after the
    // last head (a segment still open at the lane's end).
    // ---- the lane's W products, from the grouped order of the loads to the
    // order of its entries lane*W .. lane*W+W-1, through `part` (no partial
    // is staged there yet); the next tile's x gathers go out in between
    prod_t pr[W];
    products_out<DT, W>(av, xv, reinterpret_cast<prod_t *>(part), lane, pr);
    if (has_next) {
#pragma unroll
      for (int i = 0; i < W; ++i) { xv[i] = (prod_t)x[cn[i]]; av[i] = an[i]; }
    }
    products_in<DT, W>(reinterpret_cast<const prod_t *>(part), lane, pr);
    // one running sum per lane: before the lane's first head it is the part
    // of a segment opened in an earlier lane (pre); every later head closes
    // the segment summed so far, whose partial goes to its LDS slot at once.
    // At the first head the running sum is staged at that segment's slot
    // too (q - 1 = rank0 - 1, or 0 for the tile's first entry); the segment's
    // full sum overwrites it after the wave scan.  The transmitter is added
    // to the tile's first partial where that partial is read.
    Acc<DT> acc, pre;
    acc.zero();
    pre.zero();
    bool seen = false;
    int q = rank0;  // slot of the segment that the lane's next head closes, plus one
#pragma unroll
    for (int i = 0; i < W; ++i) {
      if ((hb >> i) & 1u) {
        part[q > 0 ? q - 1 : 0] = acc.value();
        if (!seen) pre = acc;
        seen = true;
        ++q;
        acc.zero();
      }
      acc.add(pr[i]);
    }
    if (!seen) pre = acc;
    // ---- wave segmented scan of the open segments (the lane's running
    // sum: its run after the last head, or all of it); carry into each lane
    Acc<DT> inc = acc;
    int f = seen ? 1 : 0;
    wave_seg_scan(inc, f);
    const Acc<DT> carry = dpp_acc<kWaveShr1, 0xf>(inc);

    // ---- the segment closed by this lane's first head: carry + pre; the
    // segment open at the tile's end (last lane): its run, or carry + pre
    // when the last lane holds no head
    if (seen && rank0 > 0) {
      Acc<DT> c = pre;
      c.prepend(carry);
      part[rank0 - 1] = c.value();
    }
    if (lane == kWave - 1) {
      Acc<DT> c = pre;
      c.prepend(carry);
      part[cnt - 1] = seen ? acc.value() : c.value();
    }
    __builtin_amdgcn_wave_barrier();

    // ---- coalesced store of the compact partials to y[start + q] (the
    // first with the transmitter added).  Two partials stay in double
    // instead: the bunch's first segment goes to the synchronizer, and the
    // last partial of a tile that ends inside row `stop` is not stored -- it
    // travels on in the transmitter to the next tile of the bunch, which
    // stores the row's sum, or, after the bunch's last tile, to the bunch's
    // tail, which stage 2 adds to the row's carries before the row's only
    // rounding to y's type.
    for (int q = lane; q < cnt; q += kWave) {
      const bool last = (q == cnt - 1);
      const int idx = start + q;
      if (!(q == 0 && start == r0) && !(last && ends_mid) && (unsigned)idx < (unsigned)m) {
        double v = part[q];
        if (q == 0) v += tx;
        y_store((y_t)v, &y[idx]);
      }
    }
    const double p0 = part[0] + tx;
    const double plast = cnt == 1 ? p0 : part[cnt - 1];
    if (start == r0) sync_v = p0;
    transmitter = ends_mid ? plast : 0.0;
    if (!has_next && ends_mid && !(cnt == 1 && start == r0) && lane == 0) a.tail_val[tb] = plast;
    __builtin_amdgcn_wave_barrier();

    // ---- dirty tile: label it for the re-arrangement, in this bunch's own
    // speculator slots (no global counter)
    if (dirty && lane == 0) {
      const int slot = __popc(dirty_bits & ((1u << t) - 1u));
      a.speculator[tb * S + slot] = make_int4(start, stop, (int)tile, 0);
    }
  }
  if (lane == 0) {
    a.sync_idx[tb] = r0;
    a.sync_val[tb] = sync_v;
    a.dirty_mask[tb] = dirty_bits;
    // a bound plan re-arranges only the bunches it listed; a dirty tile
    // anywhere else sends stage 2 to its fallback for every later call
    if (dirty_bits && !listed && a.stale) *a.stale = 1;
  }
}


// Occupancy asked of the register allocator per instance: none; every
// instance already runs at its spill-free maximum (a higher target makes the
// FP64 W = 4 instance spill).
template <int DT, int W>
constexpr int stage1_waves_per_eu() { return 1; }

template <int DT, int W, bool DEBUG>
__global__ __launch_bounds__(256)
#if SSS_WAVES_PER_EU
__attribute__((amdgpu_waves_per_eu(SSS_WAVES_PER_EU, 8)))
#else
__attribute__((amdgpu_waves_per_eu(stage1_waves_per_eu<DT, W>(), 8)))
#endif
void sss_stage1(MatCtx a) {
  extern __shared__ uint32_t lds_words[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int64_t tb = (int64_t)blockIdx.x * (blockDim.x / kWave) + wid;
  if (tb >= a.n_bunches) return;
  const int32_t brow = a.bunch_row ? a.bunch_row[tb] : -1;
  stage1_bunch<DT, W, DEBUG>(a, tb, lds_words + wid * stage1_lds_words(W, a.S), lane, brow);
}

// Plan time: the first row of every thread-bunch, the rightmost match of its
// first nonzero (Section 3.2's tile boundary search), one thread per bunch.
__device__ __forceinline__ int32_t rightmost_row(const int32_t *__restrict__ rp, int32_t m, int64_t b) {
  int32_t lo = 0, hi = m;  // rp[0] = 0 <= b
  while (lo < hi) {
    const int32_t mid = lo + (hi - lo + 1) / 2;
    if ((int64_t)rp[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void sss_bunch_rows(const int32_t *__restrict__ rp, int32_t m, int64_t SWT, int64_t n_bunches,
                               int32_t *__restrict__ out) {
  for (int64_t tb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; tb < n_bunches;
       tb += (int64_t)gridDim.x * blockDim.x)
    out[tb] = rightmost_row(rp, m, tb * SWT);
}

// Plan time: mark every bunch with a dirty tile by OR-ing `bit` into
// words[bunch * stride].  A tile is dirty exactly when an empty row r with
// row_ptr[r] = p > 0 lies in it (tile (p - 1) / WT, Section 3.2's dirty
// condition), so its bunch is (p - 1) / SWT.  Single plans mark the top bit
// of bunch_row, batch plans the last word of each bunch's bunch_info entry.
__global__ void sss_mark_dirty_bunches(const int32_t *__restrict__ rp, int32_t m, int64_t SWT,
                                       uint32_t *__restrict__ words, int stride, uint32_t bit) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = rp[r];
    if (p > 0 && p == rp[r + 1]) atomicOr(words + (p - 1) / SWT * stride, bit);
  }
}

// Plan time, batches: for global bunch g its matrix (the rightmost i with
// bunch_base[i] <= g), its first row and its index within the matrix.
__global__ void sss_batch_bunch_info(const MatCtx *__restrict__ mats, const int64_t *__restrict__ bunch_base,
                                     int32_t count, int64_t total, int4 *__restrict__ out) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = count;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo + 1) / 2;
      if (bunch_base[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    const MatCtx &a = mats[lo];
    const int64_t tb = g - bunch_base[lo];
    out[g] = make_int4(lo, rightmost_row(a.row_ptr, a.m, tb * (int64_t)a.S * a.W * kWave), (int)tb, 0);
  }
}

// Measurement aid, not part of the method: the memory floor of stage 1's
// access pattern.  Same tiling, same grouped col/val loads and the same
// one-tile-ahead prefetch as stage 1, with no row pass, no segmentation and no
// partial stores: each lane sums its products (GATHER) or its values plus
// columns (stream only) and writes one value, so the loads cannot be dropped.
template <int DT, int W, bool GATHER>
__device__ __forceinline__ double floor_bunch(const MatCtx &a, const int64_t tb, const int lane) {
  using val_t = typename VT<DT>::val_t;
  using x_t = typename VT<DT>::x_t;
  using prod_t = typename VT<DT>::prod_t;
  constexpr int WT = W * kWave;
  const int32_t *__restrict__ col = a.col;
  const val_t *__restrict__ val = static_cast<const val_t *>(a.val);
  const x_t *__restrict__ x = static_cast<const x_t *>(a.x);
  const int nnz = a.nnz, S = a.S;
  const int64_t SWT = (int64_t)S * WT;
  int cc[W];
  prod_t av[W], xv[W];
  load_tile_g<DT, W>(col, val, (int)(tb * SWT), nnz, lane, cc, av);
#pragma unroll
  for (int i = 0; i < W; ++i) xv[i] = GATHER ? (prod_t)x[cc[i]] : (prod_t)cc[i];
  double acc = 0.0;
  for (int t = 0; t < S; ++t) {
    const int64_t b64 = tb * SWT + (int64_t)t * WT;
    if (b64 >= nnz) break;
    const bool has_next = (t + 1 < S) && (b64 + WT < nnz);
    int cn[W];
    prod_t an[W];
    if (has_next) load_tile_g<DT, W>(col, val, (int)b64 + WT, nnz, lane, cn, an);
#pragma unroll
    for (int i = 0; i < W; ++i) acc += GATHER ? (double)(av[i] * xv[i]) : (double)(av[i] + xv[i]);
    if (has_next) {
#pragma unroll
      for (int i = 0; i < W; ++i) { xv[i] = GATHER ? (prod_t)x[cn[i]] : (prod_t)cn[i]; av[i] = an[i]; }
    }
  }
  return acc;
}

template <int DT, int W, bool GATHER>
__global__ __launch_bounds__(256) void sss_floor(MatCtx a, typename VT<DT>::y_t *__restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tb = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (tb >= a.n_bunches) return;
  out[tb * kWave + lane] = (typename VT<DT>::y_t)floor_bunch<DT, W, GATHER>(a, tb, lane);
}

// Many matrices in one launch per stage: the thread-bunches of all matrices
// form one nnz-balanced index space (bunch_base = prefix of the per-matrix
// bunch counts).  Stage 1 reads each bunch's matrix, first row and index
// within the matrix from the plan (found at plan time by the same
// rightmost-match search the method uses for rows); stage 2 runs that search
// over bunch_base itself.
// gfx950 (one partition) hands consecutive workgroups to its 8 XCDs in turn,
// workgroup b to XCD b mod 8, and every XCD has its own L2.
constexpr int kXcds = 8;

struct BatchArgs {
  const MatCtx *mats;
  const int64_t *bunch_base;  // [count+1]
  const int64_t *chunk_base;  // [count+1] prefix of ceil(n_bunches / 64)
  int32_t count;
  int32_t S_max;
  int64_t total_bunches;
  int64_t total_chunks;
  int64_t total_waves;        // stage-2 work items: total_chunks + n_fix + count
  int64_t n_fix;              // stage-2 re-arrangement items: the listed bunches
  const int32_t *dirty_list;  // the global bunches found at plan time to hold a dirty tile
  int32_t *stale;             // set when stage 1 finds a dirty tile in an unlisted bunch
  const int4 *bunch_info;     // per global bunch: <matrix, first row, bunch within the matrix, listed>
  // stage 1's XCD windows: the workgroups b with b mod n_windows = k take the
  // global bunches window[k] .. window[k+1]-1, in order.  n_windows is kXcds
  // (one contiguous window per XCD, holding an equal share of the nonzeros)
  // or 1 for grids of at most kXcds workgroups.
  int32_t n_windows;
  int64_t window[kXcds + 1];
};

// A global bunch's plan entry and its matrix's context, read once per
// wavefront: through the scalar unit into scalar registers, except for W = 16,
// whose register budget the scalar copy of the context pushes past the next
// occupancy step (g < 2^31: the grid is limited to that many wavefronts).
template <int W>
__device__ __forceinline__ void batch_entry(const BatchArgs &b, int64_t g, int4 &bi, MatCtx &a) {
  if constexpr (W == 16) {
    bi = b.bunch_info[g];
    a = b.mats[bi.x];
  } else {
    bi = uniform_load(b.bunch_info + uniform_i64(g));
    a = uniform_load(b.mats + bi.x);
  }
}


// The global bunch of wavefront `wid` of this workgroup in a launch of one
// wavefront per bunch over the XCD windows, or -1 past its window's end.
__device__ __forceinline__ int64_t window_bunch(const BatchArgs &b, int wid) {
  const int G = b.n_windows;
  const int k = (int)(blockIdx.x % G);
  const int64_t g = b.window[k] + (int64_t)(blockIdx.x / G) * (blockDim.x / kWave) + wid;
  return g < b.window[k + 1] ? g : -1;
}

template <int DT, int W>
__global__ __launch_bounds__(256) void sss_stage1_batch(BatchArgs b) {
  extern __shared__ uint32_t lds_words[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  uint32_t *lds_wave = lds_words + wid * stage1_lds_words(W, b.S_max);
  // One wavefront per thread-bunch, XCD-aware: workgroup blockIdx.x, which
  // runs on XCD blockIdx.x mod kXcds, takes the (blockIdx.x / kXcds)-th
  // workgroup's worth of bunches of that XCD's window, a contiguous run of
  // the global bunch space holding an eighth of the nonzeros (bunches of
  // matrices with a larger S hold more).  Each XCD then works through its
  // own run of matrices in order, and its L2 holds the x of the few matrices
  // in its window instead of those of every matrix in flight on the chip.
  // (Any placement of workgroups gives the same result; the placement only
  // decides the speed.)
  const int64_t g = window_bunch(b, wid);
  if (g < 0) return;
  int4 bi;
  MatCtx a;
  batch_entry<W>(b, g, bi, a);
  stage1_bunch<DT, W, false>(a, bi.z, lds_wave, lane, bi.w ? (int32_t)((uint32_t)bi.y | 0x80000000u) : bi.y);
}

// The same work as a persistent grid (batch_persistent plans): as many
// workgroups as stay resident, a multiple of kXcds; the workgroups with
// blockIdx.x mod kXcds = k stride over window k, one bunch per wavefront per
// step.
template <int DT, int W>
__global__ __launch_bounds__(256) void sss_stage1_batch_persistent(BatchArgs b) {
  extern __shared__ uint32_t lds_words[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  uint32_t *lds_wave = lds_words + wid * stage1_lds_words(W, b.S_max);
  const int G = b.n_windows;
  const int k = (int)(blockIdx.x % G);
  const int wpb = blockDim.x / kWave;
  const int64_t stride = (int64_t)((gridDim.x - k + G - 1) / G) * wpb;  // waves of the workgroups b mod G = k
  const int64_t hi = b.window[k + 1];
  for (int64_t g = b.window[k] + (int64_t)(blockIdx.x / G) * wpb + wid; g < hi; g += stride) {
    int4 bi;
    MatCtx a;
    batch_entry<W>(b, g, bi, a);
    stage1_bunch<DT, W, false>(a, bi.z, lds_wave, lane, bi.w ? (int32_t)((uint32_t)bi.y | 0x80000000u) : bi.y);
  }
}

// Measurement aid for the batched stage 1: its launch (one wavefront per
// bunch, the same XCD-contiguous mapping and the same per-bunch lookup) with
// floor_bunch in place of the method's work; out has 64 entries per global
// bunch.
template <int DT, int W, bool GATHER>
__global__ __launch_bounds__(256) void sss_floor_batch(BatchArgs b, typename VT<DT>::y_t *__restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int64_t g = window_bunch(b, wid);
  if (g < 0) return;
  int4 bi;
  MatCtx a;
  batch_entry<W>(b, g, bi, a);
  out[g * kWave + lane] = (typename VT<DT>::y_t)floor_bunch<DT, W, GATHER>(a, bi.z, lane);
}

// ---------------------------------------------------------------- stage 2

// (1) re-arrange the dirty tiles of thread-bunch tb: a dirty tile's partials
// 1.. sit at y[start+1..]; the k-th non-empty row strictly between start and
// stop receives partial k, the empty rows there receive 0.  Only rows strictly
// inside the tile are touched.  The partials are gathered into LDS first.
template <typename YT>
__device__ __forceinline__ void fixup_dirty(const MatCtx &a, const int64_t tb, YT *slots, const int lane) {
  const int32_t *__restrict__ rp = a.row_ptr;
  YT *y = static_cast<YT *>(a.y);
  const int WT = a.W * kWave;
  const uint32_t dm = a.dirty_mask[tb];
  const int n_dirty = __popc(dm);
  if (n_dirty == 0) return;
  // all of the bunch's speculator entries in one load: lane e holds entry e
  // (loading the slots beside the mask saves a round on bunches with dirty
  // tiles but costs more on clean ones)
  int2 ent_lane = make_int2(0, 0);
  if (lane < n_dirty) {
    const int4 s = a.speculator[tb * a.S + lane];
    ent_lane = make_int2(s.x, s.y);
  }
  for (int ent = 0; ent < n_dirty; ++ent) {
    const int start = lane_value(ent_lane.x, ent);
    const int stop = lane_value(ent_lane.y, ent);
    const int n_slots = min(stop - start - 1, WT - 1);
    // the first chunk's row bounds and the partials do not depend on each
    // other: issue both before waiting
    int r = start + 1 + lane;
    bool in = r < stop;
    int p0 = in ? rp[r] : 0, p1 = in ? rp[r + 1] : 0;
    for (int i = lane; i < n_slots; i += kWave) slots[i] = y[start + 1 + i];
    // one wavefront owns `slots` and its LDS operations execute in order:
    // only the compiler must keep the order (no wait for memory); every load
    // of y above has returned before its value reached LDS, so the stores
    // below cannot overtake them, and other tiles touch other rows
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int base = 0;
    for (int rb = start + 1; rb < stop; rb += kWave) {
      if (rb != start + 1) {
        r = rb + lane;
        in = r < stop;
        p0 = in ? rp[r] : 0;
        p1 = in ? rp[r + 1] : 0;
      }
      const bool ne = in && (p0 != p1);
      const uint64_t bal = __ballot(ne);
      const int before = __popcll(bal & ((1ull << lane) - 1ull));
      if (in) y[r] = ne ? slots[min(base + before, max(n_slots - 1, 0))] : (YT)0;
      base += __popcll(bal);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// (2) synchronizer carries for thread-bunches chunk0 .. chunk0+63 (one lane
// each): for each run of bunches whose first row is the same row r, sum their
// first-segment sums in double and write y[r] once.  Unless row r begins
// exactly where the run's first bunch begins, the part of r computed before
// the run is the tail of the bunch before the run (double), added first; y[r]
// is rounded to its type only here.  Runs of up to kShortRun bunches are
// summed by the run's first lane in bunch order, from this chunk's entries
// and the kShortRun after it staged in the wavefront's LDS (`lds`: at least
// (64 + kShortRun) * 12 bytes; register arrays for that look-ahead would cap
// the kernel's occupancy); longer runs (rows longer than kShortRun bunches)
// by the whole wavefront: coalesced loads, per-lane partial sums, then a
// fixed-shape tree over the lanes, so the rounding does not depend on timing.
template <typename YT>
__device__ __forceinline__ void fixup_carries(const MatCtx &a, const int64_t chunk0, const int lane, void *lds) {
  const int32_t *__restrict__ rp = a.row_ptr;
  YT *y = static_cast<YT *>(a.y);
  const int64_t SWT = (int64_t)a.S * a.W * kWave;
  const int64_t nb = a.n_bunches;
  const int64_t tb = chunk0 + lane;
  const bool valid = tb < nb;
  // one round of loads: this chunk's entries, the kShortRun entries after it
  // (lanes 0..kShortRun-1) and the one before it.  Entries past the last
  // bunch read as index -1, value 0.
  const int idx = valid ? a.sync_idx[tb] : -1;
  const double own_v = valid ? a.sync_val[tb] : 0.0;
  const int64_t tt = chunk0 + kWave + lane;
  const bool tail_in = lane < kShortRun && tt < nb;
  const int tail_i = tail_in ? a.sync_idx[tt] : -1;
  const double tail_v = tail_in ? a.sync_val[tt] : 0.0;
  const int before_chunk = chunk0 > 0 ? a.sync_idx[chunk0 - 1] : -1;
  double *s_val = static_cast<double *>(lds);
  int *s_idx = reinterpret_cast<int *>(s_val + kWave + kShortRun);
  s_idx[lane] = idx;
  s_val[lane] = own_v;
  if (lane < kShortRun) {
    s_idx[kWave + lane] = tail_i;
    s_val[kWave + lane] = tail_v;
  }
  // one wavefront owns `lds` and its LDS operations run in order
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int prev = wave_prev(idx, before_chunk);
  const bool head = valid && (tb == 0 || prev != idx);
  const bool is_long = head && (tb + kShortRun < nb) && (s_idx[lane + kShortRun] == idx);
  if (head && !is_long) {
    // sync_idx is non-decreasing (entries past the end read -1): the run is
    // the prefix of the next kShortRun entries equal to idx
    double sum = 0.0;
    for (int j = 0; j < kShortRun; ++j) {
      if (s_idx[lane + j] != idx) break;
      sum += s_val[lane + j];
    }
    const bool fresh = (int64_t)rp[idx] == tb * SWT;
    y[idx] = (YT)(fresh ? sum : a.tail_val[tb - 1] + sum);
  }
  uint64_t longs = __ballot(is_long);
  while (longs) {
    const int l = __ffsll((unsigned long long)longs) - 1;
    longs &= longs - 1;
    const int64_t t0 = __shfl(tb, l, kWave);
    const int ridx = __shfl(idx, l, kWave);
    double acc = 0.0;
    for (int64_t off = 0;; off += kWave) {
      const int64_t j = t0 + off + lane;
      const bool in = j < nb && a.sync_idx[j] == ridx;
      if (in) acc += a.sync_val[j];
      if (__ballot(in) != ~0ull) break;
    }
    const double total = wave_sum_tree(acc);
    if (lane == l) {
      const bool fresh = (int64_t)rp[ridx] == t0 * SWT;
      y[ridx] = (YT)(fresh ? total : a.tail_val[t0 - 1] + total);
    }
  }
  // the staged entries are read before the wavefront's next use of `lds`
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// (2b) a bound plan whose row_ptr was rewritten in place: the dirty bunches
// of chunk0 .. chunk0+63 that its list lacks, one after another (the listed
// ones have their own wavefronts).
template <typename YT>
__device__ __forceinline__ void fixup_unlisted(const MatCtx &a, const int64_t chunk0, YT *slots, const int lane,
                                               const int4 *binfo = nullptr) {
  // listed: the top bit of bunch_row (single plans), or the last word of the
  // bunch's entry in binfo (a batch's entries of this matrix)
  const int64_t tb = chunk0 + lane;
  bool todo = false;
  if (tb < a.n_bunches && a.dirty_mask[tb] != 0) todo = binfo ? binfo[tb].w == 0 : a.bunch_row[tb] >= 0;
  uint64_t todo_bits = __ballot(todo);
  while (todo_bits) {
    const int l = __ffsll((unsigned long long)todo_bits) - 1;
    todo_bits &= todo_bits - 1;
    fixup_dirty<YT>(a, chunk0 + l, slots, lane);
  }
}

// (3) rows before the first tile's start row are empty and covered by no
// tile (all rows when nnz = 0): zero them, threads first..first+stride..
template <typename YT>
__device__ __forceinline__ void fixup_leading(const MatCtx &a, const int64_t first, const int64_t stride) {
  YT *y = static_cast<YT *>(a.y);
  const int64_t r_first = a.n_bunches > 0 ? a.sync_idx[0] : a.m;
  for (int64_t r = first; r < r_first; r += stride) y[r] = (YT)0;
}

// Stage 2 of one matrix: the first ceil(n_bunches / 64) wavefronts settle the
// carries of 64 bunches each, the next n_bunches wavefronts re-arrange one
// bunch's dirty tiles each (separate wavefronts, so the two chains of
// dependent loads run side by side; a wavefront per bunch measured faster
// than a resident grid striding over the bunches, even where most bunches
// are clean); all threads share the leading rows.  The three parts write
// disjoint rows.
template <typename YT>
__global__ __launch_bounds__(1024) void sss_fixup(MatCtx a) {
  extern __shared__ unsigned char lds_raw[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  YT *slots = reinterpret_cast<YT *>(lds_raw) + (size_t)wid * a.W * kWave;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + wid;
  const int64_t n_chunks = (a.n_bunches + kWave - 1) / kWave;
  if (wave < n_chunks) {
    fixup_carries<YT>(a, wave * kWave, lane, slots);
    if (a.dirty_list && *a.stale) fixup_unlisted<YT>(a, wave * kWave, slots, lane);
  } else if (wave < n_chunks + a.n_fix) {
    fixup_dirty<YT>(a, a.dirty_list ? (int64_t)a.dirty_list[wave - n_chunks] : wave - n_chunks, slots, lane);
  }
  fixup_leading<YT>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// Stage 2 of a batch, persistent: work items 0..total_chunks-1 settle one carry
// chunk (64 bunches of one matrix) each, the next total_bunches re-arrange one
// global bunch's dirty tiles each, the last count zero one matrix's leading
// rows each.
template <typename YT>
__global__ __launch_bounds__(1024) void sss_fixup_batch(BatchArgs b) {
  extern __shared__ unsigned char lds_raw[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + wid; w < b.total_waves; w += n_waves) {
    if (w < b.total_chunks) {
      const int i = __builtin_amdgcn_readfirstlane((int)wave_rightmost(b.chunk_base, (int64_t)b.count, w, lane));
      const MatCtx a = uniform_load(b.mats + i);
      YT *slots = reinterpret_cast<YT *>(lds_raw) + (size_t)wid * a.W * kWave;
      const int64_t chunk0 = (w - uniform_load(b.chunk_base + i)) * kWave;
      fixup_carries<YT>(a, chunk0, lane, slots);
      if (*b.stale) fixup_unlisted<YT>(a, chunk0, slots, lane, b.bunch_info + uniform_load(b.bunch_base + i));
    } else if (w < b.total_chunks + b.n_fix) {
      const int64_t g = b.dirty_list[w - b.total_chunks];
      const int i = __builtin_amdgcn_readfirstlane((int)wave_rightmost(b.bunch_base, (int64_t)b.count, g, lane));
      const MatCtx a = uniform_load(b.mats + i);
      YT *slots = reinterpret_cast<YT *>(lds_raw) + (size_t)wid * a.W * kWave;
      fixup_dirty<YT>(a, g - uniform_load(b.bunch_base + i), slots, lane);
    } else {
      const MatCtx a = uniform_load(b.mats + __builtin_amdgcn_readfirstlane((int)(w - b.total_chunks - b.n_fix)));
      fixup_leading<YT>(a, lane, kWave);
    }
  }
}

template <typename YT>
__global__ void sss_fill_zero(YT *y, int64_t m) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (YT)0;
}

__global__ void sss_validate_kernel(const int32_t *rp, const int32_t *col, int64_t m, int64_t n, int64_t nnz,
                                    int *bad) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0 && (rp[0] != 0 || (int64_t)rp[m] != nnz)) atomicOr(bad, 1);
  for (int64_t i = tid; i < m; i += nt)
    if (rp[i] > rp[i + 1]) atomicOr(bad, 2);
  for (int64_t k = tid; k < nnz; k += nt)
    if (col[k] < 0 || (int64_t)col[k] >= n) atomicOr(bad, 4);
}

// ---------------------------------------------------------------- host side

int default_W(int dt) { return dt == SSS_F64 ? 8 : 16; }
int default_S(int dt) { return dt == SSS_F64 ? 5 : 2; }
constexpr int kDefaultB = 2;
// threads per stage-2 workgroup: 64 and 128 measured ~0.8 us faster than
// 256 on the 1M-row matrix (fewer waves wait on the slowest in a workgroup)
#ifndef SSS_FIXUP_THREADS
#define SSS_FIXUP_THREADS 128
#endif
constexpr int kFixupThreads = SSS_FIXUP_THREADS;
constexpr size_t kFixupLdsBytes = 64 * 1024;  // LDS of one fixup workgroup
// a stage-2 wavefront's LDS (W * 64 y values, W >= 4, y at least 4 bytes)
// also holds the carry pass's staged entries
static_assert(4 * kWave * 4 >= (kWave + kShortRun) * (sizeof(double) + sizeof(int)), "carry staging fits");
constexpr int kMaxS = 16;

bool dtype_ok(int dt) { return dt == SSS_F64 || dt == SSS_F32 || dt == SSS_BF16; }
size_t y_size(int dt) { return dt == SSS_F64 ? 8 : 4; }

int fixup_waves_per_block(int W, int dt) {
  return (int)std::max<size_t>(1, std::min<size_t>(kFixupThreads / kWave,
                                                    kFixupLdsBytes / ((size_t)W * kWave * y_size(dt))));
}

using Stage1Fn = void (*)(MatCtx);
using BatchFn = void (*)(BatchArgs);

template <int DT, int W>
Stage1Fn pick_dbg(bool dbg) { return dbg ? sss_stage1<DT, W, true> : sss_stage1<DT, W, false>; }

template <int DT>
Stage1Fn pick_w(int W, bool dbg) {
  switch (W) {
    case 4: return pick_dbg<DT, 4>(dbg);
    case 8: return pick_dbg<DT, 8>(dbg);
    case 16: return pick_dbg<DT, 16>(dbg);
    default: return nullptr;
  }
}

Stage1Fn pick_stage1(int dt, int W, bool dbg) {
  switch (dt) {
    case SSS_F64: return pick_w<SSS_F64>(W, dbg);
    case SSS_F32: return pick_w<SSS_F32>(W, dbg);
    case SSS_BF16: return pick_w<SSS_BF16>(W, dbg);
    default: return nullptr;
  }
}

template <int DT>
BatchFn pick_batch_w(int W, bool persistent) {
  switch (W) {
    case 4: return persistent ? sss_stage1_batch_persistent<DT, 4> : sss_stage1_batch<DT, 4>;
    case 8: return persistent ? sss_stage1_batch_persistent<DT, 8> : sss_stage1_batch<DT, 8>;
    case 16: return persistent ? sss_stage1_batch_persistent<DT, 16> : sss_stage1_batch<DT, 16>;
    default: return nullptr;
  }
}

BatchFn pick_stage1_batch(int dt, int W, bool persistent) {
  switch (dt) {
    case SSS_F64: return pick_batch_w<SSS_F64>(W, persistent);
    case SSS_F32: return pick_batch_w<SSS_F32>(W, persistent);
    case SSS_BF16: return pick_batch_w<SSS_BF16>(W, persistent);
    default: return nullptr;
  }
}

}  // namespace

struct sss_plan_s {
  int device = 0;
  int64_t m = 0, n = 0, nnz = 0;
  int dt = SSS_F64;
  int W = 8, S = 5, B = 2;
  int debug = 0;
  int bind_rows = 0;
  const int32_t *bound_row_ptr = nullptr;  // bind_rows plans: the row_ptr they were made for
  int64_t n_tiles = 0, n_bunches = 0;
  void *aux = nullptr;
  bool owns_aux = false;  // false: caller-provided workspace, or the static scratch
  uint32_t *dirty_mask = nullptr;
  int4 *speculator = nullptr;
  int32_t *sync_idx = nullptr;
  double *sync_val = nullptr;
  double *tail_val = nullptr;
  int32_t *bunch_row = nullptr;  // plans made with bind_rows only
  int32_t *dirty_list = nullptr; // bind_rows plans: the bunches with a dirty tile, found at plan time
  int64_t n_listed = 0;
  int32_t *stale = nullptr;      // bind_rows plans: one word, see MatCtx::stale
  int32_t *dbg_start = nullptr;
  int32_t *dbg_dirty = nullptr;
  uint32_t *dbg_heads = nullptr;
  // batch plans only
  bool batch = false;
  bool batch_persistent = false;
  BatchArgs bargs{};
  std::vector<int> mat_S;  // each matrix's tiles per thread-bunch
  int blocks1 = 0, blocks2 = 0, wpb2 = 1;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Byte offsets of a plan's auxiliary arrays in one device buffer (Section
// 3.3 sizes them: one synchronizer entry per thread-bunch, one speculator
// entry per tile), every array 256-byte aligned.
struct AuxLayout {
  int64_t n_tiles = 0, n_bunches = 0;
  size_t dmask = 0, spec = 0, sidx = 0, sval = 0, tail = 0, brow = 0, dlist = 0, stale = 0, dstart = 0, ddirty = 0,
         dheads = 0;
  size_t total = 0;
};

AuxLayout aux_layout(int64_t nnz, int W, int S, bool bind, bool debug) {
  AuxLayout L;
  const int WT = W * kWave;
  L.n_tiles = nnz > 0 ? (nnz + WT - 1) / WT : 0;
  const int64_t SWT = (int64_t)S * WT;
  L.n_bunches = nnz > 0 ? (nnz + SWT - 1) / SWT : 0;
  const size_t nt = (size_t)L.n_tiles, nb = (size_t)L.n_bunches;
  size_t off = 0;
  L.dmask = off; off = align256(off + sizeof(uint32_t) * (nb + 1));
  L.spec = off; off = align256(off + sizeof(int4) * (nb * (size_t)S + 1));
  L.sidx = off; off = align256(off + sizeof(int32_t) * (nb + 1));
  L.sval = off; off = align256(off + sizeof(double) * (nb + 1));
  L.tail = off; off = align256(off + sizeof(double) * (nb + 1));
  if (bind) {
    L.brow = off; off = align256(off + sizeof(int32_t) * (nb + 1));
    L.dlist = off; off = align256(off + sizeof(int32_t) * (nb + 1));
    L.stale = off; off = align256(off + sizeof(int32_t));
  }
  if (debug) {
    L.dstart = off; off = align256(off + sizeof(int32_t) * (nt + 1));
    L.ddirty = off; off = align256(off + sizeof(int32_t) * (nt + 1));
    L.dheads = off; off = align256(off + sizeof(uint32_t) * (nt + 1) * (size_t)(WT / 32));
  }
  L.total = off;
  return L;
}

// Point the plan's arrays into `base` (a buffer of at least L.total bytes).
void plan_bind_aux(sss_plan p, const AuxLayout &L, void *base_v) {
  char *base = static_cast<char *>(base_v);
  p->n_tiles = L.n_tiles;
  p->n_bunches = L.n_bunches;
  p->aux = base_v;
  p->dirty_mask = reinterpret_cast<uint32_t *>(base + L.dmask);
  p->speculator = reinterpret_cast<int4 *>(base + L.spec);
  p->sync_idx = reinterpret_cast<int32_t *>(base + L.sidx);
  p->sync_val = reinterpret_cast<double *>(base + L.sval);
  p->tail_val = reinterpret_cast<double *>(base + L.tail);
  p->bunch_row = p->bind_rows ? reinterpret_cast<int32_t *>(base + L.brow) : nullptr;
  p->dirty_list = p->bind_rows ? reinterpret_cast<int32_t *>(base + L.dlist) : nullptr;
  p->stale = p->bind_rows ? reinterpret_cast<int32_t *>(base + L.stale) : nullptr;
  p->dbg_start = p->debug ? reinterpret_cast<int32_t *>(base + L.dstart) : nullptr;
  p->dbg_dirty = p->debug ? reinterpret_cast<int32_t *>(base + L.ddirty) : nullptr;
  p->dbg_heads = p->debug ? reinterpret_cast<uint32_t *>(base + L.dheads) : nullptr;
}

// The plan's auxiliary buffer: the caller's workspace when given (nothing is
// allocated), else one hipMalloc owned by the plan.  Cleared on `stream`
// (stream-ordered; the caller of plan_create synchronises that stream).
int plan_alloc(sss_plan p, void *workspace, size_t workspace_bytes, hipStream_t stream) {
  const AuxLayout L = aux_layout(p->nnz, p->W, p->S, p->bind_rows != 0, p->debug != 0);
  void *base = workspace;
  if (workspace) {
    if (workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255u)) return SSS_ERR_INVALID_VALUE;
  } else {
    SSS_HIP(hipMalloc(&base, L.total));
    p->owns_aux = true;
  }
  plan_bind_aux(p, L, base);
  SSS_HIP(hipMemsetAsync(base, 0, L.total, stream));
  return SSS_OK;
}

bool misaligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) != 0; }

int check_call(sss_plan p, const int32_t *row_ptr, const int32_t *col, const void *val, const void *x, void *y) {
  if (p->m == 0) return SSS_OK;
  if (!row_ptr || !y) return SSS_ERR_INVALID_VALUE;
  if (p->nnz > 0) {
    if (!col || !val || !x) return SSS_ERR_INVALID_VALUE;
    if (misaligned(col) || misaligned(val)) return SSS_ERR_INVALID_VALUE;
  }
  // a plan whose rows were bound at plan time serves the row_ptr it was made
  // for (stage 1 also checks every bound row against row_ptr's contents and
  // searches again where one no longer holds, so y stays right even if that
  // array was rewritten in place)
  if (p->bind_rows && row_ptr != p->bound_row_ptr) return SSS_ERR_PLAN_MISMATCH;
  int dev = -1;
  SSS_HIP(hipGetDevice(&dev));
  if (dev != p->device) return SSS_ERR_PLAN_MISMATCH;
  return SSS_OK;
}

// The kernels' view of a single-matrix plan and the caller's arrays.
MatCtx plan_ctx(sss_plan p, const int32_t *row_ptr, const int32_t *col, const void *val, const void *x, void *y) {
  MatCtx a{};
  a.row_ptr = row_ptr; a.col = col; a.val = val; a.x = x; a.y = y;
  a.m = (int32_t)p->m; a.nnz = (int32_t)p->nnz; a.S = p->S; a.W = p->W;
  a.n_bunches = p->n_bunches; a.n_tiles = p->n_tiles;
  a.dirty_mask = p->dirty_mask; a.speculator = p->speculator;
  a.sync_idx = p->sync_idx; a.sync_val = p->sync_val; a.tail_val = p->tail_val;
  a.bunch_row = p->bunch_row;
  a.dirty_list = p->dirty_list;
  a.n_fix = p->dirty_list ? p->n_listed : p->n_bunches;
  a.stale = p->stale;
  a.dbg_start = p->dbg_start; a.dbg_dirty = p->dbg_dirty; a.dbg_heads = p->dbg_heads;
  return a;
}

// Stage 1: speculative execution.  (nnz = 0: y is zeroed here.)
int launch_stage1(sss_plan p, const int32_t *row_ptr, const int32_t *col, const void *val, const void *x, void *y,
                  hipStream_t stream) {
  if (p->m == 0) return SSS_OK;
  if (p->nnz == 0) {
    const int blocks = (int)std::min<int64_t>((p->m + 255) / 256, 4096);
    if (p->dt == SSS_F64)
      hipLaunchKernelGGL(sss_fill_zero<double>, dim3(blocks), dim3(256), 0, stream, (double *)y, p->m);
    else
      hipLaunchKernelGGL(sss_fill_zero<float>, dim3(blocks), dim3(256), 0, stream, (float *)y, p->m);
    SSS_HIP(hipGetLastError());
    return SSS_OK;
  }
  Stage1Fn k1 = pick_stage1(p->dt, p->W, p->debug != 0);
  if (!k1) return SSS_ERR_UNSUPPORTED;
  const MatCtx a1 = plan_ctx(p, row_ptr, col, val, x, y);
  const int64_t blocks1 = (p->n_bunches + p->B - 1) / p->B;
  const size_t lds1 = (size_t)p->B * stage1_lds_words(p->W, p->S) * sizeof(uint32_t);
  hipLaunchKernelGGL(k1, dim3((unsigned)blocks1), dim3(p->B * kWave), lds1, stream, a1);
  SSS_HIP(hipGetLastError());
  return SSS_OK;
}

// Stage 2: checking prediction (synchronizer carries, dirty-tile
// re-arrangement, leading empty rows).
int launch_stage2(sss_plan p, const int32_t *row_ptr, void *y, hipStream_t stream) {
  if (p->m == 0 || p->nnz == 0) return SSS_OK;
  const int WT = p->W * kWave;
  const MatCtx a2 = plan_ctx(p, row_ptr, nullptr, nullptr, nullptr, y);
  // one wavefront per 64 bunches (their carry runs), then one per thread-bunch
  // that can hold dirty tiles: every bunch, or a bound plan's listed ones
  const int wpb = fixup_waves_per_block(p->W, p->dt);
  const int64_t waves2 = (p->n_bunches + kWave - 1) / kWave + a2.n_fix;
  const int64_t blocks2 = std::max<int64_t>(1, (waves2 + wpb - 1) / wpb);
  const size_t lds2 = (size_t)wpb * WT * y_size(p->dt);
  if (p->dt == SSS_F64)
    hipLaunchKernelGGL(sss_fixup<double>, dim3((unsigned)blocks2), dim3(wpb * kWave), lds2, stream, a2);
  else
    hipLaunchKernelGGL(sss_fixup<float>, dim3((unsigned)blocks2), dim3(wpb * kWave), lds2, stream, a2);
  SSS_HIP(hipGetLastError());
  return SSS_OK;
}

int launch(sss_plan p, const int32_t *row_ptr, const int32_t *col, const void *val, const void *x, void *y,
           hipStream_t stream) {
  int rc = check_call(p, row_ptr, col, val, x, y);
  if (rc != SSS_OK || p->m == 0) return rc;
  rc = launch_stage1(p, row_ptr, col, val, x, y, stream);
  if (rc != SSS_OK) return rc;
  return launch_stage2(p, row_ptr, y, stream);
}

// Both stages of a batch plan: the stage-1 launch (one wavefront per
// thread-bunch of every matrix, or the persistent form), then the persistent
// stage-2 launch.
int launch_batch(sss_plan p, hipStream_t stream) {
  if (p->bargs.total_waves == 0) return SSS_OK;
  if (p->bargs.total_bunches > 0) {
    BatchFn k1 = pick_stage1_batch(p->dt, p->W, p->batch_persistent);
    if (!k1) return SSS_ERR_UNSUPPORTED;
    const size_t lds1 = (size_t)p->B * stage1_lds_words(p->W, p->bargs.S_max) * sizeof(uint32_t);
    hipLaunchKernelGGL(k1, dim3((unsigned)p->blocks1), dim3(p->B * kWave), lds1, stream, p->bargs);
    SSS_HIP(hipGetLastError());
  }
  const size_t lds2 = (size_t)p->wpb2 * p->W * kWave * y_size(p->dt);
  if (p->dt == SSS_F64)
    hipLaunchKernelGGL(sss_fixup_batch<double>, dim3((unsigned)p->blocks2), dim3(p->wpb2 * kWave), lds2, stream,
                       p->bargs);
  else
    hipLaunchKernelGGL(sss_fixup_batch<float>, dim3((unsigned)p->blocks2), dim3(p->wpb2 * kWave), lds2, stream,
                       p->bargs);
  SSS_HIP(hipGetLastError());
  return SSS_OK;
}

std::mutex g_cache_mu;
std::map<std::tuple<int, void *, int64_t, int64_t, int64_t>, sss_plan> g_cache;

// sss_validate_csr's result word: one per device, in the code object (no
// allocation per call); calls are serialised by a mutex, each waits for its
// stream before it returns
__device__ int validate_flag;
constexpr int kMaxDevices = 64;
std::mutex g_validate_mu;
int *g_validate_ptr[kMaxDevices] = {};

// sss_csr_spmv_noalloc's plan arrays (dirty masks, speculator, synchronizer,
// tails of a default double-precision plan): a static array in the code
// object, one per device, held until the process ends.  Host code never uses
// its name as an address: the device address comes from hipGetSymbolAddress,
// once per device.  Every call on a device shares it; stage 1 writes every
// entry stage 2 reads, so nothing needs clearing between calls.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

template <int DT, int W>
int launch_floor(sss_plan p, const MatCtx &a, void *out, int gather, hipStream_t stream) {
  using y_t = typename VT<DT>::y_t;
  const int64_t blocks = (p->n_bunches + p->B - 1) / p->B;
  if (gather)
    hipLaunchKernelGGL((sss_floor<DT, W, true>), dim3((unsigned)blocks), dim3(p->B * kWave), 0, stream, a,
                       static_cast<y_t *>(out));
  else
    hipLaunchKernelGGL((sss_floor<DT, W, false>), dim3((unsigned)blocks), dim3(p->B * kWave), 0, stream, a,
                       static_cast<y_t *>(out));
  SSS_HIP(hipGetLastError());
  return SSS_OK;
}

template <int DT, int W>
int launch_floor_batch(sss_plan p, void *out, int gather, hipStream_t stream) {
  using y_t = typename VT<DT>::y_t;
  if (gather)
    hipLaunchKernelGGL((sss_floor_batch<DT, W, true>), dim3((unsigned)p->blocks1), dim3(p->B * kWave), 0, stream,
                       p->bargs, static_cast<y_t *>(out));
  else
    hipLaunchKernelGGL((sss_floor_batch<DT, W, false>), dim3((unsigned)p->blocks1), dim3(p->B * kWave), 0, stream,
                       p->bargs, static_cast<y_t *>(out));
  SSS_HIP(hipGetLastError());
  return SSS_OK;
}

template <int DT>
int launch_floor_batch_w(sss_plan p, void *out, int gather, hipStream_t stream) {
  switch (p->W) {
    case 4: return launch_floor_batch<DT, 4>(p, out, gather, stream);
    case 8: return launch_floor_batch<DT, 8>(p, out, gather, stream);
    case 16: return launch_floor_batch<DT, 16>(p, out, gather, stream);
    default: return SSS_ERR_UNSUPPORTED;
  }
}

template <int DT>
int launch_floor_w(sss_plan p, const MatCtx &a, void *out, int gather, hipStream_t stream) {
  switch (p->W) {
    case 4: return launch_floor<DT, 4>(p, a, out, gather, stream);
    case 8: return launch_floor<DT, 8>(p, a, out, gather, stream);
    case 16: return launch_floor<DT, 16>(p, a, out, gather, stream);
    default: return SSS_ERR_UNSUPPORTED;
  }
}

// Stage 2 on a host core, as the paper runs it (Section 3.2, Section 3.4): the
// same three parts as the device kernel, on host arrays, one thread.
template <typename YT>
void stage2_host(sss_plan p, const int32_t *rp, YT *y, const uint32_t *dm, const int4 *spec, const int32_t *si,
                 const double *sv, const double *tv) {
  const int64_t nb = p->n_bunches;
  const int64_t WT = (int64_t)p->W * kWave, SWT = (int64_t)p->S * WT;
  // leading empty rows
  const int64_t r_first = nb > 0 ? si[0] : p->m;
  for (int64_t r = 0; r < r_first; ++r) y[r] = (YT)0;
  // dirty tiles: partial k >= 1 to the k-th non-empty row strictly inside
  std::vector<YT> slots((size_t)WT);
  for (int64_t tb = 0; tb < nb; ++tb) {
    const int n_dirty = __builtin_popcount(dm[tb]);
    for (int e = 0; e < n_dirty; ++e) {
      const int4 s = spec[tb * p->S + e];
      const int start = s.x, stop = s.y;
      const int64_t n_slots = std::min<int64_t>((int64_t)stop - start - 1, WT - 1);
      for (int64_t i = 0; i < n_slots; ++i) slots[(size_t)i] = y[start + 1 + i];
      int64_t k = 0;
      for (int64_t r = start + 1; r < stop; ++r) {
        if (rp[r] != rp[r + 1]) y[r] = slots[(size_t)std::min<int64_t>(k++, std::max<int64_t>(n_slots - 1, 0))];
        else y[r] = (YT)0;
      }
    }
  }
  // carries: runs of bunches that begin in the same row, summed in bunch
  // order after the tail of the bunch before the run (unless the row begins
  // with the run)
  for (int64_t tb = 0; tb < nb;) {
    const int idx = si[tb];
    int64_t e = tb;
    double sum = 0.0;
    while (e < nb && si[e] == idx) sum += sv[e++];
    const bool fresh = (int64_t)rp[idx] == tb * SWT;
    y[idx] = (YT)(fresh ? sum : tv[tb - 1] + sum);
    tb = e;
  }
}

}  // namespace

extern "C" {

int sss_csr_spmv_plan_workspace_size(int64_t m, int64_t n, int64_t nnz, sss_dtype dt, const sss_plan_opts *opts,
                                     size_t *bytes) {
  if (!bytes) return SSS_ERR_INVALID_VALUE;
  *bytes = 0;
  if (m < 0 || n < 0 || nnz < 0 || m > SSS_MAX_INDEX || n > SSS_MAX_INDEX || nnz > SSS_MAX_INDEX)
    return SSS_ERR_INVALID_VALUE;
  if (!dtype_ok(dt)) return SSS_ERR_UNSUPPORTED;
  sss_plan_opts o{};
  o.mode = SSS_MODE_FIXED;
  if (opts) o = *opts;
  if (o.mode != SSS_MODE_FIXED && o.mode != SSS_MODE_SELECTOR) return SSS_ERR_UNSUPPORTED;
  const bool bind = o.bind_rows && m > 0 && nnz > 0, dbg = o.debug != 0;
  size_t need = 0;
  if (o.mode == SSS_MODE_FIXED) {
    const int W = o.W ? o.W : default_W(dt), S = o.S ? o.S : default_S(dt);
    if (!(W == 4 || W == 8 || W == 16)) return SSS_ERR_UNSUPPORTED;
    if (S < 1 || S > kMaxS) return SSS_ERR_INVALID_VALUE;
    need = aux_layout(nnz, W, S, bind, dbg).total;
  } else {
    // the selector's choice is not known yet: the largest of the grid's
    // classes and the type's defaults
    need = aux_layout(nnz, default_W(dt), default_S(dt), bind, dbg).total;
    for (int c = 0; c < SSS_N_CLASSES; ++c) {
      int W = 0, S = 0;
      (void)sss_class_params(c, &W, &S);
      need = std::max(need, aux_layout(nnz, W, S, bind, dbg).total);
    }
  }
  *bytes = need;
  return SSS_OK;
}

namespace {

// Bound plans: mark every bunch with a dirty tile on the device, then list
// them on the host (bunch order) and copy the list to the plan; synchronises
// `s`.
int plan_list_dirty(sss_plan p, const int32_t *row_ptr, int64_t SWT, hipStream_t s) {
  const size_t nb = (size_t)p->n_bunches;
  const unsigned blocks = (unsigned)std::min<int64_t>((p->m + 255) / 256, 4096);
  hipLaunchKernelGGL(sss_mark_dirty_bunches, dim3(blocks), dim3(256), 0, s, row_ptr, (int32_t)p->m, SWT,
                     reinterpret_cast<uint32_t *>(p->bunch_row), 1, 0x80000000u);
  SSS_HIP(hipGetLastError());
  std::vector<int32_t> br(nb);
  SSS_HIP(hipMemcpyAsync(br.data(), p->bunch_row, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SSS_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> list;
  for (size_t tb = 0; tb < nb; ++tb)
    if (br[tb] < 0) list.push_back((int32_t)tb);
  p->n_listed = (int64_t)list.size();
  if (!list.empty()) {
    SSS_HIP(hipMemcpyAsync(p->dirty_list, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    SSS_HIP(hipStreamSynchronize(s));
  }
  return SSS_OK;
}

}  // namespace

int sss_csr_spmv_plan_create(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, sss_dtype dt,
                             const sss_plan_opts *opts, void *stream, sss_plan *out) {
  if (!out) return SSS_ERR_INVALID_VALUE;
  *out = nullptr;
  if (m < 0 || n < 0 || nnz < 0 || m > SSS_MAX_INDEX || n > SSS_MAX_INDEX || nnz > SSS_MAX_INDEX)
    return SSS_ERR_INVALID_VALUE;
  if (!dtype_ok(dt)) return SSS_ERR_UNSUPPORTED;
  sss_plan_opts o{};
  o.mode = SSS_MODE_FIXED;
  if (opts) o = *opts;
  if (o.mode != SSS_MODE_FIXED && o.mode != SSS_MODE_SELECTOR) return SSS_ERR_UNSUPPORTED;
  int W = o.W ? o.W : default_W(dt);
  int S = o.S ? o.S : default_S(dt);
  const int B = o.B ? o.B : kDefaultB;
  if (o.mode == SSS_MODE_SELECTOR && m > 0 && nnz > 0) {
    if (!row_ptr) return SSS_ERR_INVALID_VALUE;
    if (sss_selector_loaded()) {
      float f[SSS_N_FEATURES];
      int cls = 0;
      int rc = sss_csr_features(m, n, nnz, row_ptr, dt, stream, f);
      if (rc == SSS_OK) rc = sss_selector_predict(f, &cls);
      if (rc == SSS_OK) rc = sss_class_params(cls, &W, &S);
      if (rc != SSS_OK) return rc;
    } else {
      W = default_W(dt);
      S = default_S(dt);
    }
  }
  if (!(W == 4 || W == 8 || W == 16)) return SSS_ERR_UNSUPPORTED;
  if (S < 1 || S > kMaxS || B < 1 || B > 4) return SSS_ERR_INVALID_VALUE;
  if (o.bind_rows && m > 0 && nnz > 0 && !row_ptr) return SSS_ERR_INVALID_VALUE;
  if (!o.workspace && o.workspace_bytes) return SSS_ERR_INVALID_VALUE;
  sss_plan p = new sss_plan_s();
  p->m = m; p->n = n; p->nnz = nnz; p->dt = dt; p->W = W; p->S = S; p->B = B; p->debug = o.debug ? 1 : 0;
  p->bind_rows = (o.bind_rows && m > 0 && nnz > 0) ? 1 : 0;
  p->bound_row_ptr = p->bind_rows ? row_ptr : nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = SSS_OK;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { g_last_hip = e; rc = SSS_ERR_HIP; }
  if (rc == SSS_OK) rc = plan_alloc(p, o.workspace, o.workspace_bytes, s);
  if (rc == SSS_OK && p->bind_rows) {
    // each thread-bunch's first row, once for every later call
    const int64_t SWT = (int64_t)p->S * p->W * kWave;
    const unsigned blocks = (unsigned)std::min<int64_t>((p->n_bunches + 255) / 256, 65535);
    hipLaunchKernelGGL(sss_bunch_rows, dim3(blocks), dim3(256), 0, s, row_ptr, (int32_t)m, SWT, p->n_bunches,
                       p->bunch_row);
    e = hipGetLastError();
    if (e != hipSuccess) { g_last_hip = e; rc = SSS_ERR_HIP; }
    // the bunches with a dirty tile (marked in bunch_row's top bit), listed
    // in order so that stage 2 gives only them a wavefront
    if (rc == SSS_OK) rc = plan_list_dirty(p, row_ptr, SWT, s);
  }
  if (rc == SSS_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) { g_last_hip = e; rc = SSS_ERR_HIP; }
  }
  if (rc != SSS_OK) {
    if (p->owns_aux && p->aux) (void)hipFree(p->aux);
    delete p;
    return rc;
  }
  *out = p;
  return SSS_OK;
}

int sss_plan_dirty_list(sss_plan p, int32_t *host_out, int64_t cap, int64_t *n) {
  if (!p || !n || p->batch || cap < 0 || (cap > 0 && !host_out)) return SSS_ERR_INVALID_VALUE;
  if (!p->bind_rows && p->n_bunches > 0) return SSS_ERR_INVALID_VALUE;  // (no bunches: nothing to list)
  *n = p->n_listed;
  const int64_t k = std::min(cap, p->n_listed);
  if (k > 0) SSS_HIP(hipMemcpy(host_out, p->dirty_list, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost));
  return SSS_OK;
}

int sss_csr_spmv_execute(sss_plan p, const int32_t *row_ptr, const int32_t *col, const void *val, const void *x,
                         void *y, void *stream) {
  if (!p || p->batch) return SSS_ERR_INVALID_VALUE;
  return launch(p, row_ptr, col, val, x, y, static_cast<hipStream_t>(stream));
}

int sss_csr_spmv_stage1(sss_plan p, const int32_t *row_ptr, const int32_t *col, const void *val, const void *x,
                        void *y, void *stream) {
  if (!p || p->batch) return SSS_ERR_INVALID_VALUE;
  const int rc = check_call(p, row_ptr, col, val, x, y);
  if (rc != SSS_OK || p->m == 0) return rc;
  return launch_stage1(p, row_ptr, col, val, x, y, static_cast<hipStream_t>(stream));
}

int sss_floor_probe(sss_plan p, const int32_t *col, const void *val, const void *x, void *out, int gather,
                    void *stream) {
  if (!p || p->batch) return SSS_ERR_INVALID_VALUE;
  if (p->m == 0 || p->nnz == 0) return SSS_OK;
  if (!col || !val || !out || (gather && !x)) return SSS_ERR_INVALID_VALUE;
  if (misaligned(col) || misaligned(val)) return SSS_ERR_INVALID_VALUE;
  int dev = -1;
  SSS_HIP(hipGetDevice(&dev));
  if (dev != p->device) return SSS_ERR_PLAN_MISMATCH;
  MatCtx a{};
  a.col = col; a.val = val; a.x = x;
  a.m = (int32_t)p->m; a.nnz = (int32_t)p->nnz; a.S = p->S; a.W = p->W;
  a.n_bunches = p->n_bunches; a.n_tiles = p->n_tiles;
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (p->dt) {
    case SSS_F64: return launch_floor_w<SSS_F64>(p, a, out, gather, s);
    case SSS_F32: return launch_floor_w<SSS_F32>(p, a, out, gather, s);
    case SSS_BF16: return launch_floor_w<SSS_BF16>(p, a, out, gather, s);
    default: return SSS_ERR_UNSUPPORTED;
  }
}

int sss_csr_spmv_stage2(sss_plan p, const int32_t *row_ptr, void *y, void *stream) {
  if (!p || p->batch) return SSS_ERR_INVALID_VALUE;
  if (p->m == 0) return SSS_OK;
  if (!row_ptr || !y) return SSS_ERR_INVALID_VALUE;
  if (p->bind_rows && row_ptr != p->bound_row_ptr) return SSS_ERR_PLAN_MISMATCH;
  int dev = -1;
  SSS_HIP(hipGetDevice(&dev));
  if (dev != p->device) return SSS_ERR_PLAN_MISMATCH;
  return launch_stage2(p, row_ptr, y, static_cast<hipStream_t>(stream));
}

int sss_csr_spmv(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col, const double *val,
                 const double *x, double *y, void *stream) {
  if (m < 0 || n < 0 || nnz < 0) return SSS_ERR_INVALID_VALUE;
  if (m == 0) return SSS_OK;
  int dev = 0;
  SSS_HIP(hipGetDevice(&dev));
  sss_plan p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto key = std::make_tuple(dev, stream, m, n, nnz);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      p = it->second;
    } else {
      const int rc = sss_csr_spmv_plan_create(m, n, nnz, row_ptr, SSS_F64, nullptr, stream, &p);
      if (rc != SSS_OK) return rc;
      g_cache[key] = p;
    }
  }
  return launch(p, row_ptr, col, val, x, y, static_cast<hipStream_t>(stream));
}

int sss_csr_spmv_noalloc(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                         const double *val, const double *x, double *y, void *stream) {
  if (m < 0 || n < 0 || nnz < 0 || m > SSS_MAX_INDEX || n > SSS_MAX_INDEX || nnz > SSS_MAX_INDEX)
    return SSS_ERR_INVALID_VALUE;
  if (m == 0) return SSS_OK;
  const AuxLayout L = aux_layout(nnz, default_W(SSS_F64), default_S(SSS_F64), false, false);
  if (L.total > kScratchBytes) return SSS_ERR_TOO_LARGE;
  int dev = -1;
  SSS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SSS_ERR_UNSUPPORTED;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *ptr = nullptr;
      SSS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
      g_scratch_ptr[dev] = ptr;
    }
    base = g_scratch_ptr[dev];
  }
  sss_plan_s p;
  p.device = dev;
  p.m = m; p.n = n; p.nnz = nnz; p.dt = SSS_F64;
  p.W = default_W(SSS_F64); p.S = default_S(SSS_F64); p.B = kDefaultB;
  plan_bind_aux(&p, L, base);
  return launch(&p, row_ptr, col, val, x, y, static_cast<hipStream_t>(stream));
}

int sss_csr_spmv_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (g_cache.empty()) return SSS_OK;
  int rc = SSS_OK, cur = -1;
  const hipError_t eg = hipGetDevice(&cur);
  for (auto &kv : g_cache) {
    // each plan is destroyed with its own device current
    hipError_t e = hipSetDevice(kv.second->device);
    int r = e == hipSuccess ? sss_plan_destroy(kv.second) : SSS_ERR_HIP;
    if (e != hipSuccess) g_last_hip = e;
    if (rc == SSS_OK) rc = r;
  }
  g_cache.clear();
  if (eg == hipSuccess && cur >= 0) (void)hipSetDevice(cur);
  return rc;
}

int sss_csr_spmv_stage2_host(sss_plan p, const int32_t *row_ptr, void *y) {
  if (!p || p->batch) return SSS_ERR_INVALID_VALUE;
  if (p->m == 0 || p->nnz == 0) return SSS_OK;
  if (!row_ptr || !y) return SSS_ERR_INVALID_VALUE;
  const size_t nb = (size_t)p->n_bunches;
  std::vector<uint32_t> dm(nb);
  std::vector<int4> spec(nb * (size_t)p->S);
  std::vector<int32_t> si(nb);
  std::vector<double> sv(nb), tv(nb);
  SSS_HIP(hipDeviceSynchronize());
  SSS_HIP(hipMemcpy(dm.data(), p->dirty_mask, nb * sizeof(uint32_t), hipMemcpyDeviceToHost));
  SSS_HIP(hipMemcpy(spec.data(), p->speculator, spec.size() * sizeof(int4), hipMemcpyDeviceToHost));
  SSS_HIP(hipMemcpy(si.data(), p->sync_idx, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
  SSS_HIP(hipMemcpy(sv.data(), p->sync_val, nb * sizeof(double), hipMemcpyDeviceToHost));
  SSS_HIP(hipMemcpy(tv.data(), p->tail_val, nb * sizeof(double), hipMemcpyDeviceToHost));
  if (p->dt == SSS_F64)
    stage2_host(p, row_ptr, static_cast<double *>(y), dm.data(), spec.data(), si.data(), sv.data(), tv.data());
  else
    stage2_host(p, row_ptr, static_cast<float *>(y), dm.data(), spec.data(), si.data(), sv.data(), tv.data());
  return SSS_OK;
}

int sss_plan_destroy(sss_plan p) {
  if (!p) return SSS_OK;
  int rc = SSS_OK;
  // hipFree waits for the device's outstanding work before it frees (so a
  // replay of the plan's graph has ended before the graph goes); a
  // caller-provided workspace stays with the caller
  // every resource is released even when an earlier release fails; the
  // first failure is the one reported
  hipError_t first = hipSuccess;
  auto release = [&first](hipError_t e) { if (first == hipSuccess) first = e; };
  if (p->owns_aux && p->aux) release(hipFree(p->aux));
  if (p->graph_exec) release(hipGraphExecDestroy(p->graph_exec));
  if (p->graph) release(hipGraphDestroy(p->graph));
  if (p->capture_stream) release(hipStreamDestroy(p->capture_stream));
  if (first != hipSuccess) { g_last_hip = first; rc = SSS_ERR_HIP; }
  delete p;
  return rc;
}

int sss_batch_plan_create(int count, const sss_csr_desc *mats, sss_dtype dt, const sss_plan_opts *opts,
                          void *stream, sss_plan *out) {
  if (!out || count < 0 || (count > 0 && !mats)) return SSS_ERR_INVALID_VALUE;
  *out = nullptr;
  if (!dtype_ok(dt)) return SSS_ERR_UNSUPPORTED;
  sss_plan_opts o{};
  o.mode = SSS_MODE_FIXED;
  if (opts) o = *opts;
  if (o.mode != SSS_MODE_FIXED && o.mode != SSS_MODE_SELECTOR) return SSS_ERR_UNSUPPORTED;
  int W = o.W ? o.W : default_W(dt);
  const int S = o.S ? o.S : default_S(dt);
  const int B = o.B ? o.B : kDefaultB;
  if (!(W == 4 || W == 8 || W == 16)) return SSS_ERR_UNSUPPORTED;
  if (S < 1 || S > kMaxS || B < 1 || B > 4 || o.debug) return SSS_ERR_INVALID_VALUE;
  // SELECTOR mode: every matrix's S from its class scores, W shared
  std::vector<int> sel_S;
  if (o.mode == SSS_MODE_SELECTOR && count > 0 && sss_selector_loaded()) {
    for (int i = 0; i < count; ++i)
      if (mats[i].m < 0 || mats[i].n < 0 || mats[i].nnz < 0 || mats[i].m > SSS_MAX_INDEX ||
          mats[i].n > SSS_MAX_INDEX || mats[i].nnz > SSS_MAX_INDEX || (mats[i].m > 0 && !mats[i].row_ptr))
        return SSS_ERR_INVALID_VALUE;
    std::vector<float> scores((size_t)count * SSS_N_CLASSES, 0.f);
    double w_votes[17] = {};
    // a matrix is scored with its own row-structure features but the size
    // features of the whole launch: the batch's bunches share one grid, so
    // how well a tile schedule fills the device depends on the total work,
    // not on the one matrix
    double tot_m = 0, tot_n = 0, tot_nnz = 0;
    for (int i = 0; i < count; ++i) { tot_m += (double)mats[i].m; tot_n += (double)mats[i].n; tot_nnz += (double)mats[i].nnz; }
    for (int i = 0; i < count; ++i) {
      const sss_csr_desc &d = mats[i];
      if (d.m == 0 || d.nnz == 0) continue;
      float f[SSS_N_FEATURES];
      int rc = sss_csr_features(d.m, d.n, d.nnz, d.row_ptr, dt, stream, f);
      f[0] = (float)std::log2(tot_m + 1.0);
      f[1] = (float)std::log2(tot_n + 1.0);
      f[2] = (float)std::log2(tot_nnz + 1.0);
      if (rc == SSS_OK) rc = sss_selector_scores(f, &scores[(size_t)i * SSS_N_CLASSES]);
      if (rc != SSS_OK) return rc;
      const float *z = &scores[(size_t)i * SSS_N_CLASSES];
      const int best = (int)(std::max_element(z, z + SSS_N_CLASSES) - z);
      int Wc = 0, Sc = 0;
      (void)sss_class_params(best, &Wc, &Sc);
      w_votes[Wc] += (double)d.nnz;
    }
    if (!o.W) W = w_votes[4] > w_votes[8] && w_votes[4] > w_votes[16] ? 4 : (w_votes[16] > w_votes[8] ? 16 : 8);
    sel_S.assign((size_t)count, S);
    for (int i = 0; i < count; ++i) {
      if (mats[i].m == 0 || mats[i].nnz == 0) continue;
      const float *z = &scores[(size_t)i * SSS_N_CLASSES];
      float best = -INFINITY;
      for (int c = 0; c < SSS_N_CLASSES; ++c) {
        int Wc = 0, Sc = 0;
        (void)sss_class_params(c, &Wc, &Sc);
        if (Wc == W && z[c] > best) { best = z[c]; sel_S[(size_t)i] = Sc; }
      }
    }
  }
  const int WT = W * kWave;
  std::vector<MatCtx> ctx((size_t)count);
  std::vector<int64_t> bb((size_t)count + 1, 0), cb((size_t)count + 1, 0), sb((size_t)count + 1, 0);
  int s_max = 1;
  int64_t tot_m = 0, tot_n = 0, tot_nnz = 0, tot_tiles = 0;
  for (int i = 0; i < count; ++i) {
    const sss_csr_desc &d = mats[i];
    if (d.m < 0 || d.n < 0 || d.nnz < 0 || d.m > SSS_MAX_INDEX || d.n > SSS_MAX_INDEX || d.nnz > SSS_MAX_INDEX)
      return SSS_ERR_INVALID_VALUE;
    if (d.m > 0 && (!d.row_ptr || !d.y)) return SSS_ERR_INVALID_VALUE;
    if (d.nnz > 0 && (!d.col || !d.val || !d.x || misaligned(d.col) || misaligned(d.val))) return SSS_ERR_INVALID_VALUE;
    const int Si = !sel_S.empty() ? sel_S[(size_t)i] : (d.S ? d.S : S);
    if (Si < 1 || Si > kMaxS) return SSS_ERR_INVALID_VALUE;
    s_max = std::max(s_max, Si);
    const int64_t nb = (d.m > 0 && d.nnz > 0) ? (d.nnz + (int64_t)Si * WT - 1) / ((int64_t)Si * WT) : 0;
    MatCtx &c = ctx[(size_t)i];
    c.row_ptr = d.row_ptr; c.col = d.col; c.val = d.val; c.x = d.x; c.y = d.y;
    c.m = (int32_t)d.m; c.nnz = (int32_t)d.nnz; c.S = Si; c.W = W; c.n_bunches = nb;
    c.n_tiles = d.nnz > 0 ? (d.nnz + WT - 1) / WT : 0;
    c.dbg_start = nullptr; c.dbg_dirty = nullptr; c.dbg_heads = nullptr;
    bb[(size_t)i + 1] = bb[(size_t)i] + nb;
    cb[(size_t)i + 1] = cb[(size_t)i] + (nb + kWave - 1) / kWave;
    sb[(size_t)i + 1] = sb[(size_t)i] + nb * Si;
    tot_m += d.m; tot_n += d.n; tot_nnz += d.nnz; tot_tiles += c.n_tiles;
  }
  const int64_t nb_all = bb[(size_t)count], spec_all = sb[(size_t)count];
  // global bunch indices are listed as int32 (the dirty list): more bunches
  // than that is beyond any batch that fits in memory
  if (nb_all > INT32_MAX) return SSS_ERR_INVALID_VALUE;
  size_t off = 0;
  const size_t o_mats = off; off = align256(off + sizeof(MatCtx) * (size_t)std::max(count, 1));
  const size_t o_bb = off; off = align256(off + sizeof(int64_t) * ((size_t)count + 1));
  const size_t o_cb = off; off = align256(off + sizeof(int64_t) * ((size_t)count + 1));
  const size_t o_dm = off; off = align256(off + sizeof(uint32_t) * (size_t)(nb_all + 1));
  const size_t o_sp = off; off = align256(off + sizeof(int4) * (size_t)(spec_all + 1));
  const size_t o_si = off; off = align256(off + sizeof(int32_t) * (size_t)(nb_all + 1));
  const size_t o_sv = off; off = align256(off + sizeof(double) * (size_t)(nb_all + 1));
  const size_t o_tv = off; off = align256(off + sizeof(double) * (size_t)(nb_all + 1));
  const size_t o_bi = off; off = align256(off + sizeof(int4) * (size_t)(nb_all + 1));
  const size_t o_dl = off; off = align256(off + sizeof(int32_t) * (size_t)(nb_all + 1));
  const size_t o_st = off; off = align256(off + sizeof(int32_t));

  sss_plan p = new sss_plan_s();
  p->batch = true; p->dt = dt; p->W = W; p->S = S; p->B = B; p->batch_persistent = o.batch_persistent != 0;
  p->mat_S.resize((size_t)count);
  for (int i = 0; i < count; ++i) p->mat_S[(size_t)i] = ctx[(size_t)i].S;
  p->m = tot_m; p->n = tot_n; p->nnz = tot_nnz; p->n_tiles = tot_tiles; p->n_bunches = nb_all;
  auto fail = [&](hipError_t e) {
    g_last_hip = e;
    if (p->aux) (void)hipFree(p->aux);
    delete p;
    return SSS_ERR_HIP;
  };
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return fail(e);
  e = hipMalloc(&p->aux, off);
  if (e != hipSuccess) { p->aux = nullptr; return fail(e); }
  p->owns_aux = true;
  e = hipMemsetAsync(p->aux, 0, off, s);
  if (e != hipSuccess) return fail(e);
  char *base = static_cast<char *>(p->aux);
  for (int i = 0; i < count; ++i) {
    MatCtx &c = ctx[(size_t)i];
    c.dirty_mask = reinterpret_cast<uint32_t *>(base + o_dm) + bb[(size_t)i];
    c.speculator = reinterpret_cast<int4 *>(base + o_sp) + sb[(size_t)i];
    c.sync_idx = reinterpret_cast<int32_t *>(base + o_si) + bb[(size_t)i];
    c.sync_val = reinterpret_cast<double *>(base + o_sv) + bb[(size_t)i];
    c.tail_val = reinterpret_cast<double *>(base + o_tv) + bb[(size_t)i];
    c.stale = reinterpret_cast<int32_t *>(base + o_st);
  }
  // host arrays stay alive until the stream synchronisation below
  if (count > 0)
    e = hipMemcpyAsync(base + o_mats, ctx.data(), sizeof(MatCtx) * (size_t)count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + o_bb, bb.data(), sizeof(int64_t) * ((size_t)count + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + o_cb, cb.data(), sizeof(int64_t) * ((size_t)count + 1), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(e);
  BatchArgs &ba = p->bargs;
  ba.mats = reinterpret_cast<const MatCtx *>(base + o_mats);
  ba.bunch_base = reinterpret_cast<const int64_t *>(base + o_bb);
  ba.chunk_base = reinterpret_cast<const int64_t *>(base + o_cb);
  ba.count = count;
  ba.S_max = s_max;
  ba.total_bunches = nb_all;
  ba.total_chunks = cb[(size_t)count];
  ba.dirty_list = reinterpret_cast<const int32_t *>(base + o_dl);
  ba.stale = reinterpret_cast<int32_t *>(base + o_st);
  // every global bunch's matrix, first row and index within the matrix, once
  // for all calls (the descriptors, and so the row pointers, are bound to the plan)
  int4 *binfo = reinterpret_cast<int4 *>(base + o_bi);
  ba.bunch_info = binfo;
  if (nb_all > 0) {
    const unsigned blocks = (unsigned)std::min<int64_t>((nb_all + 255) / 256, 65535);
    hipLaunchKernelGGL(sss_batch_bunch_info, dim3(blocks), dim3(256), 0, s, ba.mats, ba.bunch_base, count, nb_all,
                       binfo);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
    // the bunches with a dirty tile, marked in their bunch_info entries
    for (int i = 0; i < count && e == hipSuccess; ++i) {
      const MatCtx &c = ctx[(size_t)i];
      if (c.n_bunches == 0) continue;
      const unsigned mb = (unsigned)std::min<int64_t>(((int64_t)c.m + 255) / 256, 4096);
      hipLaunchKernelGGL(sss_mark_dirty_bunches, dim3(mb), dim3(256), 0, s, c.row_ptr, c.m, (int64_t)c.S * WT,
                         reinterpret_cast<uint32_t *>(binfo + bb[(size_t)i]) + 3, 4, 1u);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return fail(e);
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(e);
  // list them in order, so that stage 2 gives only them a work item
  std::vector<int32_t> dlist;
  if (nb_all > 0) {
    std::vector<int4> bi_host((size_t)nb_all);
    e = hipMemcpy(bi_host.data(), binfo, sizeof(int4) * (size_t)nb_all, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(e);
    for (int64_t g = 0; g < nb_all; ++g)
      if (bi_host[(size_t)g].w) dlist.push_back((int32_t)g);
    if (!dlist.empty()) {
      e = hipMemcpy(base + o_dl, dlist.data(), sizeof(int32_t) * dlist.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) return fail(e);
    }
  }
  ba.n_fix = (int64_t)dlist.size();
  ba.total_waves = ba.total_chunks + ba.n_fix + count;
  // stage 2's persistent grid: as many workgroups as stay resident on the device
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) return fail(e);
  int per_cu2 = 0;
  p->wpb2 = fixup_waves_per_block(W, dt);
  const size_t lds2 = (size_t)p->wpb2 * WT * y_size(dt);
  const void *k2 = dt == SSS_F64 ? reinterpret_cast<const void *>(sss_fixup_batch<double>)
                                 : reinterpret_cast<const void *>(sss_fixup_batch<float>);
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, k2, p->wpb2 * kWave, lds2);
  if (e != hipSuccess) return fail(e);
  // stage 1: B bunches per workgroup, the count rounded up to a multiple of
  // kXcds so that every XCD gets an equal contiguous run (the extra
  // wavefronts find no bunch and exit); persistent: as many workgroups as
  // stay resident, a multiple of kXcds
  int64_t wgs1 = std::max<int64_t>(1, (nb_all + B - 1) / B);
  if (p->batch_persistent) {
    int per_cu1 = 0;
    const size_t lds1 = (size_t)B * stage1_lds_words(W, s_max) * sizeof(uint32_t);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu1, reinterpret_cast<const void *>(pick_stage1_batch(dt, W, true)), B * kWave, lds1);
    if (e != hipSuccess) return fail(e);
    wgs1 = std::min<int64_t>(wgs1, (int64_t)cus * std::max(per_cu1, 1));
    if (wgs1 > kXcds) wgs1 -= wgs1 % kXcds;
  }
  // the XCD windows: one per XCD when the grid has more than kXcds
  // workgroups, each a contiguous run of global bunches that holds an equal
  // share of the nonzeros (a bunch holds S W 64 of its matrix's, the last
  // one of a matrix fewer), so that matrices with a larger S do not load
  // their XCD more; else a single window
  ba.n_windows = wgs1 > kXcds ? kXcds : 1;
  for (int k = 0; k <= kXcds; ++k) ba.window[k] = nb_all;
  ba.window[0] = 0;
  if (ba.n_windows == kXcds) {
    int k = 1;
    int64_t before = 0;  // nonzeros of the matrices before matrix i
    for (int i = 0; i < count && k < kXcds; ++i) {
      const MatCtx &c = ctx[(size_t)i];
      const int64_t swt = (int64_t)c.S * WT;
      while (k < kXcds && c.n_bunches > 0 && before + c.nnz >= tot_nnz * k / kXcds) {
        const int64_t j = std::min<int64_t>(c.n_bunches, (tot_nnz * k / kXcds - before + swt / 2) / swt);
        ba.window[k] = std::max(ba.window[k - 1], bb[(size_t)i] + j);
        ++k;
      }
      before += c.nnz;
    }
    int64_t per = 0;  // workgroups per XCD: enough for its largest window
    for (int w = 0; w < kXcds; ++w) per = std::max(per, (ba.window[w + 1] - ba.window[w] + B - 1) / B);
    if (!p->batch_persistent) wgs1 = kXcds * std::max<int64_t>(per, 1);
  }
  if (wgs1 > INT32_MAX) {  // more bunches than a grid holds: beyond any batch that fits in memory
    (void)hipFree(p->aux);
    delete p;
    return SSS_ERR_INVALID_VALUE;
  }
  p->blocks1 = (int)wgs1;
  p->blocks2 = (int)std::max<int64_t>(
      1, std::min<int64_t>((ba.total_waves + p->wpb2 - 1) / p->wpb2, (int64_t)cus * std::max(per_cu2, 1)));
  *out = p;
  return SSS_OK;
}

int sss_batch_execute(sss_plan p, void *stream) {
  if (!p || !p->batch) return SSS_ERR_INVALID_VALUE;
  int dev = -1;
  SSS_HIP(hipGetDevice(&dev));
  if (dev != p->device) return SSS_ERR_PLAN_MISMATCH;
  return launch_batch(p, static_cast<hipStream_t>(stream));
}

int sss_batch_graph_launch(sss_plan p, void *stream) {
  if (!p || !p->batch) return SSS_ERR_INVALID_VALUE;
  int dev = -1;
  SSS_HIP(hipGetDevice(&dev));
  if (dev != p->device) return SSS_ERR_PLAN_MISMATCH;
  if (!p->graph_exec) {
    if (!p->capture_stream) SSS_HIP(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
    SSS_HIP(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
    const int rc = launch_batch(p, p->capture_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->capture_stream, &g);
    if (rc != SSS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) { g_last_hip = e; return SSS_ERR_HIP; }
    const hipError_t ei = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      // nothing is kept: the next call captures again
      (void)hipGraphDestroy(g);
      p->graph_exec = nullptr;
      g_last_hip = ei;
      return SSS_ERR_HIP;
    }
    p->graph = g;
  }
  SSS_HIP(hipGraphLaunch(p->graph_exec, static_cast<hipStream_t>(stream)));
  return SSS_OK;
}

int sss_batch_floor_probe(sss_plan p, void *out, int gather, void *stream) {
  if (!p || !p->batch) return SSS_ERR_INVALID_VALUE;
  if (p->batch_persistent) return SSS_ERR_UNSUPPORTED;  // the probe mirrors the default launch
  if (p->bargs.total_bunches == 0) return SSS_OK;
  if (!out) return SSS_ERR_INVALID_VALUE;
  int dev = -1;
  SSS_HIP(hipGetDevice(&dev));
  if (dev != p->device) return SSS_ERR_PLAN_MISMATCH;
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (p->dt) {
    case SSS_F64: return launch_floor_batch_w<SSS_F64>(p, out, gather, s);
    case SSS_F32: return launch_floor_batch_w<SSS_F32>(p, out, gather, s);
    case SSS_BF16: return launch_floor_batch_w<SSS_BF16>(p, out, gather, s);
    default: return SSS_ERR_UNSUPPORTED;
  }
}

int sss_batch_plan_schedule(sss_plan p, int count, int *W, int *S) {
  if (!p || !p->batch || count != (int)p->mat_S.size()) return SSS_ERR_INVALID_VALUE;
  if (W) *W = p->W;
  if (S) std::copy(p->mat_S.begin(), p->mat_S.end(), S);
  return SSS_OK;
}

int sss_plan_info(sss_plan p, int *W, int *S, int *B, int64_t *n_tiles, int64_t *n_bunches) {
  if (!p) return SSS_ERR_INVALID_VALUE;
  if (W) *W = p->W;
  if (S) *S = p->S;
  if (B) *B = p->B;
  if (n_tiles) *n_tiles = p->n_tiles;
  if (n_bunches) *n_bunches = p->n_bunches;
  return SSS_OK;
}

int sss_plan_shape(sss_plan p, int64_t *m, int64_t *n, int64_t *nnz, sss_dtype *dt) {
  if (!p || p->batch) return SSS_ERR_INVALID_VALUE;
  if (m) *m = p->m;
  if (n) *n = p->n;
  if (nnz) *nnz = p->nnz;
  if (dt) *dt = static_cast<sss_dtype>(p->dt);
  return SSS_OK;
}

int sss_validate_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col, void *stream) {
  if (m < 0 || n < 0 || nnz < 0) return SSS_ERR_INVALID_VALUE;
  if (!row_ptr || (nnz > 0 && !col)) return SSS_ERR_INVALID_VALUE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = -1;
  SSS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SSS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_validate_mu);
  if (!g_validate_ptr[dev]) {
    void *ptr = nullptr;
    SSS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(validate_flag)));
    g_validate_ptr[dev] = static_cast<int *>(ptr);
  }
  int *d_bad = g_validate_ptr[dev];
  int rc = SSS_OK;
  hipError_t e = hipMemsetAsync(d_bad, 0, sizeof(int), s);
  if (e == hipSuccess) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((std::max(m, nnz) + 255) / 256, 4096));
    hipLaunchKernelGGL(sss_validate_kernel, dim3(blocks), dim3(256), 0, s, row_ptr, col, m, n, nnz, d_bad);
    e = hipGetLastError();
  }
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { g_last_hip = e; rc = SSS_ERR_HIP; }
  if (rc == SSS_OK && bad) rc = SSS_ERR_INVALID_CSR;
  return rc;
}

int sss_plan_debug_size(sss_plan p, size_t *bytes) {
  if (!p || !bytes) return SSS_ERR_INVALID_VALUE;
  const size_t wpt = (size_t)p->W * kWave / 32;
  *bytes = 4 * sizeof(int64_t) + (size_t)p->n_tiles * (2 * sizeof(int32_t) + wpt * sizeof(uint32_t)) +
           (size_t)p->n_tiles * 4 * sizeof(int32_t) + (size_t)p->n_bunches * (sizeof(int32_t) + 2 * sizeof(double));
  return SSS_OK;
}

int sss_plan_debug_dump(sss_plan p, void *host_buf, size_t bytes) {
  if (p && p->batch) return SSS_ERR_INVALID_VALUE;
  size_t need = 0;
  int rc = sss_plan_debug_size(p, &need);
  if (rc != SSS_OK) return rc;
  if (!host_buf || bytes < need) return SSS_ERR_INVALID_VALUE;
  SSS_HIP(hipDeviceSynchronize());
  std::memset(host_buf, 0, need);
  const int64_t nt = p->n_tiles, nb = p->n_bunches;
  const int64_t wpt = (int64_t)p->W * kWave / 32;
  // the per-bunch speculator segments, packed into one list in bunch order
  std::vector<uint32_t> dmask((size_t)nb);
  std::vector<int4> spec((size_t)(nb * p->S));
  if (nb > 0) {
    SSS_HIP(hipMemcpy(dmask.data(), p->dirty_mask, nb * sizeof(uint32_t), hipMemcpyDeviceToHost));
    SSS_HIP(hipMemcpy(spec.data(), p->speculator, nb * p->S * sizeof(int4), hipMemcpyDeviceToHost));
  }
  std::vector<int4> packed;
  for (int64_t b = 0; b < nb; ++b)
    for (int i = 0; i < __builtin_popcount(dmask[(size_t)b]); ++i) packed.push_back(spec[(size_t)(b * p->S + i)]);
  int64_t *hdr = static_cast<int64_t *>(host_buf);
  hdr[0] = nt; hdr[1] = nb; hdr[2] = (int64_t)packed.size(); hdr[3] = wpt;
  char *cur = reinterpret_cast<char *>(hdr + 4);
  if (p->debug && nt > 0) {
    SSS_HIP(hipMemcpy(cur, p->dbg_start, nt * sizeof(int32_t), hipMemcpyDeviceToHost));
    SSS_HIP(hipMemcpy(cur + nt * sizeof(int32_t), p->dbg_dirty, nt * sizeof(int32_t), hipMemcpyDeviceToHost));
    SSS_HIP(hipMemcpy(cur + 2 * nt * sizeof(int32_t), p->dbg_heads, nt * wpt * sizeof(uint32_t),
                      hipMemcpyDeviceToHost));
  }
  cur += nt * (2 * sizeof(int32_t) + wpt * sizeof(uint32_t));
  if (!packed.empty()) std::memcpy(cur, packed.data(), packed.size() * sizeof(int4));
  cur += nt * 4 * sizeof(int32_t);
  if (nb > 0) {
    SSS_HIP(hipMemcpy(cur, p->sync_idx, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
    SSS_HIP(hipMemcpy(cur + nb * sizeof(int32_t), p->sync_val, nb * sizeof(double), hipMemcpyDeviceToHost));
    SSS_HIP(hipMemcpy(cur + nb * (sizeof(int32_t) + sizeof(double)), p->tail_val, nb * sizeof(double),
                      hipMemcpyDeviceToHost));
  }
  return SSS_OK;
}

const char *sss_status_string(int status) {
  switch (status) {
    case SSS_OK: return "ok";
    case SSS_ERR_INVALID_VALUE: return "invalid value";
    case SSS_ERR_UNSUPPORTED: return "unsupported dtype or parameters";
    case SSS_ERR_PLAN_MISMATCH: return "plan does not match the call";
    case SSS_ERR_HIP: return "HIP runtime error";
    case SSS_ERR_INVALID_CSR: return "malformed CSR matrix";
    case SSS_ERR_TOO_LARGE: return "matrix too large for the static scratch of sss_csr_spmv_noalloc";
    default: return "unknown status";
  }
}

const char *sss_last_hip_error(void) { return hipGetErrorString(g_last_hip); }

const char *sss_version(void) { return "sss-spmv 0.1 gfx950"; }

}  // extern "C"
