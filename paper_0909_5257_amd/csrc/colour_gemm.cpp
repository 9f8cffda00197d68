// Colour quadratic form of the paper's eq. (color-averaged-amplitude) for many amplitude
// vectors: q_r = sum_{a,b} J_ra N_ab J_rb^* with N real symmetric.  With the real and
// imaginary parts of J as separate real rows x (2R rows of K), q_r is the sum of x^T N x over
// the two rows of r, i.e. the GEMM Y = X N followed by a row-wise dot (section 3.3 blames this
// step for much of the GPU time).
//
// For K <= 128 the contraction runs in hand-written gfx950 kernels that read J from HBM once,
// convert it in registers and keep N in LDS (no work space, nothing staged in HBM):
//   HEGET_COLOUR_FP64       v_mfma_f64_16x16x4_f64,
//   HEGET_COLOUR_FP32       v_mfma_f32_16x16x4_f32 (float32 operands, float32 accumulate),
//   HEGET_COLOUR_BF16X3     v_mfma_f32_16x16x32_bf16 three times per product: x and N split
//                           into bf16 high and low parts, x N ~ xh Nh + xh Nl + xl Nh,
//                           float32 accumulate,
//   HEGET_COLOUR_FP64_VALU  float64 vector FMAs (the same sum without the matrix cores).
// Symmetry halves the matrix work: with 16-colour blocks, q = sum_{A<=B} x_A^T W_AB x_B where
// W_AB = 2 N_AB above the diagonal and N_AA on it.  Each MFMA tile computes
// Y^T[m][t] = sum_a W[a][m] x_t[a] for 16 output colours m and 16 rows t; the inner colours of
// one instruction are ordered so that each lane already holds, as its MFMA operand, exactly the
// four x values its four output elements must be dotted with, so the row dot needs no data
// movement.  The dot is accumulated in float64 against the float64 x in every mode.
// Larger K falls back to a plain library GEMM (rocBLAS) plus a row-dot kernel.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <type_traits>
#include <mutex>

#include "heget.h"

namespace {

std::mutex g_mutex;
std::map<int, rocblas_handle> g_handles;

rocblas_handle handle_for(int dev) {
  auto it = g_handles.find(dev);
  if (it != g_handles.end()) return it->second;
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
  g_handles[dev] = h;
  // keep freed work space in the device's stream-ordered pool between calls instead of
  // handing it back to the HIP runtime at every synchronisation (re-mapping gigabytes per call)
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t keep = uint64_t(16) << 30;     // up to 16 GiB stays cached
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  return h;
}

__global__ void to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// Columns of length K (one per real row) -> columns of length 3K holding [hi; hi; lo].
__global__ void split_cols_bf16(const double* __restrict__ x, __hip_bfloat16* __restrict__ y, int k, int64_t cols,
                                int lo_block) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)k * cols) return;
  const int64_t c = i / k;
  const int a = (int)(i - c * k);
  const double v = x[i];
  const __hip_bfloat16 hi = __float2bfloat16((float)v);
  const __hip_bfloat16 lo = __float2bfloat16((float)(v - (double)__bfloat162float(hi)));
  __hip_bfloat16* col = y + c * (int64_t)(3 * k);
  for (int blk = 0; blk < 3; ++blk) col[blk * k + a] = (blk == lo_block) ? lo : hi;
}

// N (K x K, column-major, symmetric) -> [Nh | Nl | Nh] (K x 3K column-major).
__global__ void split_matrix_bf16(const double* __restrict__ n, __hip_bfloat16* __restrict__ y, int k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k * k) return;
  const double v = n[i];
  const __hip_bfloat16 hi = __float2bfloat16((float)v);
  const __hip_bfloat16 lo = __float2bfloat16((float)(v - (double)__bfloat162float(hi)));
  y[i] = hi;
  y[k * k + i] = lo;
  y[2 * k * k + i] = hi;
}

// One wave per row: the 64 lanes read consecutive elements of the row (coalesced) and the
// partial sums are combined with a butterfly over the wave.
template <class T>
__global__ __launch_bounds__(256) void row_dot(const double* __restrict__ x, const T* __restrict__ y, int k,
                                               int64_t rows, double* __restrict__ q) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;                      // whole waves leave together
  const double* xr = x + r * 2 * k;
  const T* yr = y + r * 2 * k;
  double s = 0.0;
  for (int a = lane; a < 2 * k; a += 64) s += xr[a] * (double)yr[a];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) q[r] = s;
}

inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- hand-written kernels (K <= 128)

constexpr int kMaxK = 128;          // colours: at most 8 blocks of 16
constexpr int kNB = kMaxK / 16;
constexpr int kWaves = 4;           // waves per workgroup
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// Symmetrised block weight: W_ab = 2 N_ab if block(a) < block(b), N_ab if the blocks are equal,
// 0 below the block diagonal or outside the K x K matrix.
__device__ __forceinline__ double wsym(const double* __restrict__ n, int k, int a, int b) {
  if (a >= k || b >= k) return 0.0;
  const int ba = a >> 4, bb = b >> 4;
  if (ba > bb) return 0.0;
  const double v = n[(int64_t)a * k + b];
  return ba < bb ? 2.0 * v : v;
}

// Wave tile: 16 real rows.  Lane l works on row t = l % 16 and lane group g = l / 16.  The A and B
// operands of the 16x16x4 instructions put A[i][k] in lane i + 16 k and B[k][j] in lane j + 16 k.
// x[A][s] = x_t[16 A + 4 g + s]: the MFMA B operand of inner step s of block A (inner index g of
// the instruction is colour 16 A + 4 g + s) and, for output block B = A, the four values that
// the lane's output elements D[i] = Y^T[16 B + 4 g + i][t] are dotted with.
__device__ __forceinline__ void load_tile(const double* __restrict__ x, int k, int64_t nreal, int64_t r0, int lane,
                                          double (&xv)[kNB][4]) {
  const int64_t row = r0 + (lane & 15);
  const int g = lane >> 4;
  const bool ok = row < nreal;
  const double* src = x + row * k;
#pragma unroll
  for (int a = 0; a < kNB; ++a)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int c = 16 * a + 4 * g + s;
      xv[a][s] = (ok && c < k) ? src[c] : 0.0;
    }
}

// Sum the row partials of the four lane groups, add the two real rows of each amplitude row and
// write q for the tile's 8 amplitude rows.
__device__ __forceinline__ void finish_tile(double dot, int lane, int64_t r0, int64_t nreal, double* __restrict__ q) {
  dot += __shfl_xor(dot, 16, 64);
  dot += __shfl_xor(dot, 32, 64);
  dot += __shfl_xor(dot, 1, 64);
  const int64_t row = r0 + lane;
  if (lane < 16 && !(lane & 1) && row < nreal) q[row >> 1] = dot;
}

// float64 / float32 operands, 16x16x4 instructions.
template <class T>
__global__ __launch_bounds__(64 * kWaves) void qf_mfma4(int k, const double* __restrict__ nmat,
                                                          const double* __restrict__ x, int64_t nreal,
                                                          double* __restrict__ q) {
  // W in A-operand order: per block pair (A <= B) and inner step s, the 64 lane values
  __shared__ T ws[kNB * (kNB + 1) / 2 * 4 * 64];
  const int nb = (k + 15) >> 4;
  const int npair = nb * (nb + 1) / 2;
  for (int e = threadIdx.x; e < npair * 256; e += 64 * kWaves) {
    const int p = e >> 8, s = (e >> 6) & 3, l = e & 63;
    int bb = 0;
    while ((bb + 1) * (bb + 2) / 2 <= p) ++bb;
    const int ba = p - bb * (bb + 1) / 2;
    // output row i of the instruction is colour 16 B + m(i): the float32 instruction leaves row i in
    // lane group i / 4, register i % 4, and the float64 one in lane group i % 4, register i / 4, so
    // for float64 the rows are transposed (m(i) = 4 (i % 4) + i / 4) to put the same colours
    // 16 B + 4 g + r in lane group g, register r in both cases
    const int i = l & 15;
    const int m = sizeof(T) == 8 ? 4 * (i & 3) + (i >> 2) : i;
    ws[e] = (T)wsym(nmat, k, 16 * ba + 4 * (l >> 4) + s, 16 * bb + m);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ntiles = (nreal + 15) >> 4;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles; tile += (int64_t)gridDim.x * kWaves) {
    const int64_t r0 = tile * 16;
    double xv[kNB][4];
    load_tile(x, k, nreal, r0, lane, xv);
    double dot = 0.0;
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      if (b < nb) {
        using V = typename std::conditional<sizeof(T) == 8, d4_t, f4_t>::type;
        V acc = {0, 0, 0, 0};
#pragma unroll
        for (int a = 0; a <= b; ++a)
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const T w = ws[((b * (b + 1) / 2 + a) * 4 + s) * 64 + lane];
            if constexpr (sizeof(T) == 8)
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(w, xv[a][s], acc, 0, 0, 0);
            else
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w, (float)xv[a][s], acc, 0, 0, 0);
          }
#pragma unroll
        for (int i = 0; i < 4; ++i) dot += (double)acc[i] * xv[b][i];
      }
    }
    finish_tile(dot, lane, r0, nreal, q);
  }
}

__device__ __forceinline__ void split_bf16(double v, __bf16& hi, __bf16& lo) {
  const float f = (float)v;
  hi = (__bf16)f;
  lo = (__bf16)(f - (float)hi);
}

// bf16 hi/lo split, three 16x16x32 instructions per product.  Inner index 8 g + j of an
// instruction over 32-colour block A2 is colour 16 (2 A2) + 4 g + j for j < 4 and
// 16 (2 A2 + 1) + 4 g + (j - 4) otherwise, so the B operand is (x[2 A2][0..3], x[2 A2 + 1][0..3]).
__global__ __launch_bounds__(64 * kWaves) void qf_mfma_bf16x3(int k, const double* __restrict__ nmat,
                                                              const double* __restrict__ x, int64_t nreal,
                                                              double* __restrict__ q) {
  // per (output block B, inner 32-block A2 <= B / 2): [hi | lo][lane] of 8 bf16
  constexpr int kPairs = (kNB / 2) * (kNB / 2 + 1);      // sum over B of (B / 2 + 1) = 20 for 8 blocks
  __shared__ bf8_t ws[kPairs * 2 * 64];
  const int nb = (k + 15) >> 4;
  for (int e = threadIdx.x; e < kPairs * 64; e += 64 * kWaves) {
    const int p = e >> 6, l = e & 63;
    // pair p -> (B, A2) in the order B = 0.., A2 = 0..B/2
    int bb = 0, base = 0;
    while (base + bb / 2 + 1 <= p) {
      base += bb / 2 + 1;
      ++bb;
    }
    const int a2 = p - base;
    bf8_t hi, lo;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int a = 16 * (2 * a2 + (j >> 2)) + 4 * (l >> 4) + (j & 3);
      const double w = bb < nb ? wsym(nmat, k, a, 16 * bb + (l & 15)) : 0.0;
      __bf16 h, o;
      split_bf16(w, h, o);
      hi[j] = h;
      lo[j] = o;
    }
    ws[(p * 2) * 64 + l] = hi;
    ws[(p * 2 + 1) * 64 + l] = lo;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ntiles = (nreal + 15) >> 4;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles; tile += (int64_t)gridDim.x * kWaves) {
    const int64_t r0 = tile * 16;
    double xv[kNB][4];
    load_tile(x, k, nreal, r0, lane, xv);
    bf8_t xh[kNB / 2], xl[kNB / 2];
#pragma unroll
    for (int a2 = 0; a2 < kNB / 2; ++a2)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 h, o;
        split_bf16(xv[2 * a2 + (j >> 2)][j & 3], h, o);
        xh[a2][j] = h;
        xl[a2][j] = o;
      }
    double dot = 0.0;
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      if (b < nb) {
        f4_t acc = {0, 0, 0, 0};
        const int base = (b / 2) * (b / 2 + 1) + (b & 1) * (b / 2 + 1);   // pairs before output block b
#pragma unroll
        for (int a2 = 0; a2 <= b / 2; ++a2) {
          const bf8_t wh = ws[((base + a2) * 2) * 64 + lane];
          const bf8_t wl = ws[((base + a2) * 2 + 1) * 64 + lane];
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xh[a2], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xl[a2], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, xh[a2], acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) dot += (double)acc[i] * xv[b][i];
      }
    }
    finish_tile(dot, lane, r0, nreal, q);
  }
}

// float64 on the vector ALUs.  The symmetric weights of q_t = sum_a x_ta (N_aa x_ta + 2 sum_{b > a}
// N_ab x_tb) are staged in LDS once per workgroup, in 8-row blocks j laid out as [b - 8 j][8] for
// b >= 8 j (the upper block triangle, 0 below the diagonal and outside K x K), so each wave reads 8
// consecutive weights with broadcast loads.  The workgroup stages 64 real rows transposed in LDS (one
// per lane); the row blocks are dealt to the waves in the order 0, 1, ..., W-1, W-1, ..., 0, W, ...
// (their lengths fall with the block index).
constexpr int kValuW = (kMaxK / 8) * 8 * kMaxK - 8 * 8 * (kMaxK / 8) * (kMaxK / 8 - 1) / 2;   // doubles

__global__ __launch_bounds__(64 * kWaves) void qf_valu_f64(int k, const double* __restrict__ nmat,
                                                           const double* __restrict__ x, int64_t nreal,
                                                           double* __restrict__ q) {
  __shared__ double xs[kMaxK][64];
  __shared__ double wl[kValuW];
  __shared__ double part[kWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kp = (k + 7) & ~7;
  const int nblk = kp >> 3;
  // block j starts at 8 * sum_{j' < j} (kp - 8 j') = 8 j kp - 32 j (j - 1)
  for (int j = 0; j < nblk; ++j) {
    const int off = 8 * j * kp - 32 * j * (j - 1), len = 8 * (kp - 8 * j);
    for (int e = threadIdx.x; e < len; e += 64 * kWaves) {
      const int a = 8 * j + (e & 7), b = 8 * j + (e >> 3);
      wl[off + e] = (a < k && b < k && b >= a) ? (b == a ? 1.0 : 2.0) * nmat[(int64_t)a * k + b] : 0.0;
    }
  }
  const int64_t ntiles = (nreal + 63) >> 6;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * 64;
    const int64_t nrow = nreal - r0 < 64 ? nreal - r0 : 64;
    const double* src = x + r0 * k;
    // wave w copies rows w, w + W, ...: its lanes read consecutive colours of one row
    for (int t = wave; t < 64; t += kWaves)
      for (int c = lane; c < kp; c += 64) xs[c][t] = (t < nrow && c < k) ? src[(int64_t)t * k + c] : 0.0;
    __syncthreads();
    double acc = 0.0;
    for (int j = 0; j < nblk; ++j) {
      const int round = j / kWaves, pos = j - round * kWaves;
      if ((round & 1 ? kWaves - 1 - pos : pos) != wave) continue;
      const int a0 = 8 * j;
      const double* wj = wl + 8 * j * kp - 32 * j * (j - 1);
      double tr[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) tr[i] = 0.0;
      for (int b = a0; b < kp; ++b) {
        const double xb = xs[b][lane];
        const double* wb = wj + 8 * (b - a0);
#pragma unroll
        for (int i = 0; i < 8; ++i) tr[i] += wb[i] * xb;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) acc += xs[a0 + i][lane] * tr[i];
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += part[w][lane];
      t += __shfl_xor(t, 1, 64);
      if (!(lane & 1) && lane < nrow) q[(r0 + lane) >> 1] = t;
    }
    __syncthreads();
  }
}

hipError_t launch_hand_written(int k, const double* nmat, const double* jamp, int64_t rows, heget_colour_mode mode,
                               double* q, hipStream_t s) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t nreal = 2 * rows;
  if (mode == HEGET_COLOUR_FP64_VALU) {
    const int64_t tiles = (nreal + 63) / 64;
    const unsigned grid = (unsigned)std::min<int64_t>(tiles, (int64_t)cus * 2);
    hipLaunchKernelGGL(qf_valu_f64, dim3(grid), dim3(64 * kWaves), 0, s, k, nmat, jamp, nreal, q);
    return hipGetLastError();
  }
  const int64_t tiles = (nreal + 15) / 16;
  const unsigned grid = (unsigned)std::min<int64_t>((tiles + kWaves - 1) / kWaves, (int64_t)cus * 8);
  if (mode == HEGET_COLOUR_FP64)
    hipLaunchKernelGGL(qf_mfma4<double>, dim3(grid), dim3(64 * kWaves), 0, s, k, nmat, jamp, nreal, q);
  else if (mode == HEGET_COLOUR_FP32)
    hipLaunchKernelGGL(qf_mfma4<float>, dim3(grid), dim3(64 * kWaves), 0, s, k, nmat, jamp, nreal, q);
  else
    hipLaunchKernelGGL(qf_mfma_bf16x3, dim3(grid), dim3(64 * kWaves), 0, s, k, nmat, jamp, nreal, q);
  return hipGetLastError();
}

}  // namespace

extern "C" heget_status heget_colour_quadratic_form(int k, const double* nmat, const double* jamp, int64_t rows,
                                                    heget_colour_mode mode, double* q, void* stream) {
  if (k <= 0 || rows < 0 || rows >= (int64_t(1) << 30)) return HEGET_E_INVALID_ARG;
  if (mode != HEGET_COLOUR_FP64 && mode != HEGET_COLOUR_FP32 && mode != HEGET_COLOUR_BF16X3 &&
      mode != HEGET_COLOUR_FP64_VALU)
    return HEGET_E_INVALID_ARG;
  if (mode == HEGET_COLOUR_FP64_VALU && k > kMaxK) return HEGET_E_INVALID_ARG;
  if (rows == 0) return HEGET_OK;
  if (!nmat || !jamp || !q) return HEGET_E_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (k <= kMaxK) return launch_hand_written(k, nmat, jamp, rows, mode, q, s) == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;
  // larger colour spaces: library GEMM (rocBLAS) into a stream-ordered work space, then the row dot
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HEGET_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_mutex);
  rocblas_handle h = handle_for(dev);
  if (!h || rocblas_set_stream(h, s) != rocblas_status_success) return HEGET_E_DEVICE;
  const int64_t cols = 2 * rows;          // real rows of X = columns of X^T (K x 2R, column-major)
  const int64_t nx = cols * k;
  heget_status st = HEGET_OK;
  if (mode == HEGET_COLOUR_FP64) {
    double* y = nullptr;
    if (hipMallocAsync(&y, sizeof(double) * nx, s) != hipSuccess) return HEGET_E_OUT_OF_MEMORY;
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, k, (rocblas_int)cols, k, &one, nmat, k,
                      jamp, k, &zero, y, k) != rocblas_status_success)
      st = HEGET_E_DEVICE;
    else
      hipLaunchKernelGGL(row_dot<double>, dim3(blocks(rows, 4)), dim3(256), 0, s, jamp, y, k, rows, q);
    (void)hipFreeAsync(y, s);
  } else if (mode == HEGET_COLOUR_FP32) {
    float *x32 = nullptr, *n32 = nullptr, *y = nullptr;
    if (hipMallocAsync(&x32, sizeof(float) * nx, s) != hipSuccess) return HEGET_E_OUT_OF_MEMORY;
    if (hipMallocAsync(&n32, sizeof(float) * k * k, s) != hipSuccess) {
      (void)hipFreeAsync(x32, s);
      return HEGET_E_OUT_OF_MEMORY;
    }
    if (hipMallocAsync(&y, sizeof(float) * nx, s) != hipSuccess) {
      (void)hipFreeAsync(x32, s);
      (void)hipFreeAsync(n32, s);
      return HEGET_E_OUT_OF_MEMORY;
    }
    hipLaunchKernelGGL(to_f32, dim3(blocks(nx, 256)), dim3(256), 0, s, jamp, x32, nx);
    hipLaunchKernelGGL(to_f32, dim3(blocks(k * k, 256)), dim3(256), 0, s, nmat, n32, (int64_t)k * k);
    const float one = 1.0f, zero = 0.0f;
    if (rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_none, k, (rocblas_int)cols, k, &one, n32, k, x32,
                      k, &zero, y, k) != rocblas_status_success)
      st = HEGET_E_DEVICE;
    else
      hipLaunchKernelGGL(row_dot<float>, dim3(blocks(rows, 4)), dim3(256), 0, s, jamp, y, k, rows, q);
    (void)hipFreeAsync(x32, s);
    (void)hipFreeAsync(n32, s);
    (void)hipFreeAsync(y, s);
  } else {
    __hip_bfloat16 *xb = nullptr, *nb = nullptr;
    float* y = nullptr;
    if (hipMallocAsync(&xb, sizeof(__hip_bfloat16) * 3 * nx, s) != hipSuccess) return HEGET_E_OUT_OF_MEMORY;
    if (hipMallocAsync(&nb, sizeof(__hip_bfloat16) * 3 * k * k, s) != hipSuccess) {
      (void)hipFreeAsync(xb, s);
      return HEGET_E_OUT_OF_MEMORY;
    }
    if (hipMallocAsync(&y, sizeof(float) * nx, s) != hipSuccess) {
      (void)hipFreeAsync(xb, s);
      (void)hipFreeAsync(nb, s);
      return HEGET_E_OUT_OF_MEMORY;
    }
    // [Nh | Nl | Nh] . [Xh; Xh; Xl] = Nh Xh + Nl Xh + Nh Xl
    hipLaunchKernelGGL(split_cols_bf16, dim3(blocks(nx, 256)), dim3(256), 0, s, jamp, xb, k, cols, 2);
    hipLaunchKernelGGL(split_matrix_bf16, dim3(blocks(k * k, 256)), dim3(256), 0, s, nmat, nb, k);
    const float one = 1.0f, zero = 0.0f;
    if (rocblas_gemm_ex(h, rocblas_operation_none, rocblas_operation_none, k, (rocblas_int)cols, 3 * k, &one, nb,
                        rocblas_datatype_bf16_r, k, xb, rocblas_datatype_bf16_r, 3 * k, &zero, y,
                        rocblas_datatype_f32_r, k, y, rocblas_datatype_f32_r, k, rocblas_datatype_f32_r,
                        rocblas_gemm_algo_standard, 0, 0) != rocblas_status_success)
      st = HEGET_E_DEVICE;
    else
      hipLaunchKernelGGL(row_dot<float>, dim3(blocks(rows, 4)), dim3(256), 0, s, jamp, y, k, rows, q);
    (void)hipFreeAsync(xb, s);
    (void)hipFreeAsync(nb, s);
    (void)hipFreeAsync(y, s);
  }
  if (st == HEGET_OK && hipGetLastError() != hipSuccess) st = HEGET_E_DEVICE;
  return st;
}
