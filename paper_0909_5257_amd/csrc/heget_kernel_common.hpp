// Pieces shared by every generated process kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Per-process descriptor emitted by the generator and registered with the library.
struct heget_proc_desc {
  const char* spec;              // normalised process string, e.g. "g g > g g g g"
  int n_ext;                     // external legs
  int n_diagrams;                // Feynman diagrams (four-gluon vertex counted per colour piece)
  int n_colours;                 // colour-basis size K
  int n_helicities;              // helicity configurations that are not structural zeros
  int n_helicities_all;          // 2^n_ext
  int colour_table_len;          // doubles in colour_table (0: the kernel holds N inline)
  const double* colour_table;    // blocked upper-triangular N for the LDS colour sum
  const long long* colour_num;   // exact N_ab = num/den, row-major K*K, includes 1/(n_a n_b)
  const long long* colour_den;
  long long flops_per_event;     // floating-point operations of one event, counted by the generator
  hipError_t (*launch)(int precision, const double* mom, int64_t n, double* out,
                       const double* colour_table_dev, double scale, hipStream_t stream);
};

namespace heget {

// Read one event's momenta (AoS, n legs x (E, px, py, pz)) with 16-byte loads.
template <int NEXT>
__device__ __forceinline__ void load_momenta(const double* __restrict__ mom, int64_t ev, double (&pm)[NEXT][4]) {
  const double2* src = reinterpret_cast<const double2*>(mom + ev * (int64_t)(NEXT * 4));
#pragma unroll
  for (int i = 0; i < NEXT; ++i) {
    double2 a = src[2 * i], b = src[2 * i + 1];
    pm[i][0] = a.x;
    pm[i][1] = a.y;
    pm[i][2] = b.x;
    pm[i][3] = b.y;
  }
}

// Copy the momenta through an empty asm so that values derived from them are
// recomputed inside the helicity loop instead of being hoisted out of it
// (hoisting every subset momentum would hold hundreds of registers live).
template <int NEXT>
__device__ __forceinline__ void opaque_copy(const double (&pm)[NEXT][4], double (&pp)[NEXT][4]) {
#pragma unroll
  for (int i = 0; i < NEXT; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double v = pm[i][j];
      asm volatile("" : "+v"(v));
      pp[i][j] = v;
    }
}

// Colour quadratic form sum_{a,b} J_a N_ab J_b^* for J held in LDS as
// jl[a][lane] = (Re J_a, Im J_a).  N is real symmetric; the table holds
// M_ab = N_ab (b > a), N_aa / 2 (b = a), 0 (b < a) in blocks of B rows laid
// out as [K/B][K][B] so that the B row values of one column are contiguous
// and wave-uniform (scalar loads).  Result: 2 sum_a sum_b M_ab J_a . J_b.
template <int K, int B>
__device__ __forceinline__ double colour_sum_lds(double2 (*jl)[64], int lane, const double* __restrict__ cmat) {
  static_assert(K % B == 0, "colour block must divide the basis size");
  double q = 0.0;
#pragma unroll 1
  for (int blk = 0; blk < K / B; ++blk) {
    const int a0 = blk * B;
    const double* m = cmat + (int64_t)blk * K * B;
    double tr[B], ti[B];
#pragma unroll
    for (int a = 0; a < B; ++a) {
      tr[a] = 0.0;
      ti[a] = 0.0;
    }
#pragma unroll 2
    for (int b = a0; b < K; ++b) {
      const double2 jb = jl[b][lane];
#pragma unroll
      for (int a = 0; a < B; ++a) {
        const double mab = m[b * B + a];
        tr[a] += mab * jb.x;
        ti[a] += mab * jb.y;
      }
    }
#pragma unroll
    for (int a = 0; a < B; ++a) {
      const double2 ja = jl[a0 + a][lane];
      q += ja.x * tr[a] + ja.y * ti[a];
    }
  }
  return 2.0 * q;
}

}  // namespace heget
