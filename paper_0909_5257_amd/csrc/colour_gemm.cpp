// Colour quadratic form as a GEMM: q_r = sum_{a,b} J_ra N_ab J_rb^* for many rows.
//
// The paper's eq. (color-averaged-amplitude) contracts every colour-basis
// amplitude vector with the real symmetric colour matrix.  Written with the
// real and imaginary parts of J as separate rows X (2R x K), it is
// Y = X N followed by a row-wise dot q_r = X_2r . Y_2r + X_2r+1 . Y_2r+1.
// Three precisions of the contraction are offered for study:
//   HEGET_COLOUR_FP64    float64 GEMM,
//   HEGET_COLOUR_FP32    float32 GEMM on the matrix cores,
//   HEGET_COLOUR_BF16X3  bf16 split X = Xh + Xl, N = Nh + Nl, with
//                        Y ~ Xh Nh + Xh Nl + Xl Nh in one bf16 GEMM over the
//                        concatenated inner dimension 3K, float32 accumulate.
// The GEMMs are plain library GEMMs (rocBLAS); the split and the dot are
// kernels here.  The dot always accumulates in float64 against the float64 X.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <map>
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

}  // namespace

extern "C" heget_status heget_colour_quadratic_form(int k, const double* nmat, const double* jamp, int64_t rows,
                                                    heget_colour_mode mode, double* q, void* stream) {
  if (k <= 0 || rows < 0 || rows > (int64_t(1) << 31) / 2) return HEGET_E_INVALID_ARG;
  if (mode != HEGET_COLOUR_FP64 && mode != HEGET_COLOUR_FP32 && mode != HEGET_COLOUR_BF16X3)
    return HEGET_E_INVALID_ARG;
  if (rows == 0) return HEGET_OK;
  if (!nmat || !jamp || !q) return HEGET_E_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
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
