// Pieces shared by every generated process kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "heget_device.hpp"

// Per-process descriptor emitted by the generator and registered with the library.
struct heget_proc_desc {
  const char* spec;              // normalised process string, e.g. "g g > g g g g"
  int n_ext;                     // external legs
  int n_diagrams;                // Feynman diagrams (four-gluon vertex counted per colour piece)
  int n_colours;                 // colour-basis size K
  int n_helicities;              // helicity configurations that are not structural zeros
  int n_helicities_all;          // 2^n_ext
  int colour_table_len;          // doubles in colour_table (0: the kernel holds N inline)
  const double* colour_table;    // blocked upper-triangular W for the LDS colour sum
  const long long* colour_num;   // exact N_ab = num/den, row-major K*K, includes 1/(n_a n_b)
  const long long* colour_den;
  long long flops_per_event[2];  // floating-point operations one event executes (float64, mixed), incl. recomputation
  long long algo_flops_per_event;  // the same with every shared current counted once (roofline numerator)
  // hel == nullptr: sum over helicities; otherwise one helicity bit pattern per event, and with
  // perm != nullptr launch slot i evaluates event perm[i]
  hipError_t (*launch)(int precision, const double* mom, const int* hel, const int* perm, int64_t n,
                       double* out, const double* colour_table_dev, double scale, hipStream_t stream);
  int n_patterns;                // quark-chirality patterns of the sampled-helicity kernels
  const int* helicity_pattern;   // per bit pattern h: its chirality pattern, -1 for a structural zero
  int k_reduced;                 // dimension K' of the reduced colour vector y the kernels accumulate
  int n_slots;                   // evaluated helicity configurations (leg 0 at +1, no structural zeros)
  const int* slot_helicity;      // helicity bit pattern of each evaluated configuration, loop order
  const long long* red_num;      // y = M J, M = red_num / red_den (K' x K, row-major)
  const long long* red_den;
  const long long* w_num;        // Q = y^H W y, W = w_num / w_den (K' x K', row-major)
  const long long* w_den;
  // test-hook kernels (nullptr if not generated): gauge leg substitution eps -> k/E (-1: none) and,
  // with jamp != nullptr, y of every evaluated configuration as float64 [n][n_slots][K'][2]
  hipError_t (*launch_hook)(int precision, const double* mom, int64_t n, double* out, const double* colour_table_dev,
                            double scale, int gauge, double* jamp, hipStream_t stream);
  long long max_launch_events;   // events one kernel launch covers (larger batches run in slices)
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

// Opaque copies: the compiler may not assume the copy equals its source, so
// values computed from a copy in one group of amplitudes are never merged with
// values computed in another group.  Components known to vanish for external
// wavefunctions (eps^0, Im eps^3) are passed through unchanged.
__device__ __forceinline__ void opaque(double& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void opaque(float& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ int opaque_int(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ __forceinline__ mom4<double> fresh(const mom4<double>& p) {
  mom4<double> q = p;
  opaque(q.e); opaque(q.x); opaque(q.y); opaque(q.z);
  return q;
}
template <class R> __device__ __forceinline__ vec4<R> fresh(const vec4<R>& v) {
  vec4<R> w = v;
  opaque(w.c1.re); opaque(w.c1.im); opaque(w.c2.re); opaque(w.c2.im); opaque(w.c3.re);
  return w;
}
template <class R> __device__ __forceinline__ wsp<R> fresh(const wsp<R>& f) {
  wsp<R> g = f;
  opaque(g.s0.re); opaque(g.s0.im); opaque(g.s1.re); opaque(g.s1.im);
  return g;
}
__device__ __forceinline__ mom4<double> neg(const mom4<double>& p) { return {-p.e, -p.x, -p.y, -p.z}; }

// Relaxed workgroup-scope float64 add into LDS (native LDS float64 atomic on gfx950).
__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Share of the colour quadratic form computed by one wave, for a colour vector held in LDS as
// yl[a][0|1][lane]: the wave takes the row blocks listed in blocks (blocks[0] = their count; the
// generator deals the blocks of the upper triangle to the waves longest first).  The table holds
// M_ab = W_ab (b > a), W_aa / 2 (b = a), 0 (b < a) in blocks of B rows laid out as [K/B][K][B] so that
// the B row values of one column are contiguous and wave-uniform (scalar loads).  The column loop is
// unrolled by U so that the loads of U columns are in flight together.  Result: 2 sum over the
// wave's rows of sum_b M_ab (Re y_a Re y_b + Im y_a Im y_b).
template <int K, int B, int U>
__device__ __forceinline__ double colour_sum_lds_part(double (*yl)[2][64], int lane, const int* __restrict__ blocks,
                                                      const double* __restrict__ cmat) {
  static_assert(K % B == 0, "colour block must divide the colour dimension");
  double q = 0.0;
  const int nblk = blocks[0];
#pragma unroll 1
  for (int i = 1; i <= nblk; ++i) {
    const int blk = blocks[i];
    const int a0 = blk * B;
    const double* m = cmat + (int64_t)blk * K * B;
    double tr[B], ti[B];
#pragma unroll
    for (int a = 0; a < B; ++a) {
      tr[a] = 0.0;
      ti[a] = 0.0;
    }
#pragma unroll U
    for (int b = a0; b < K; ++b) {
      const double jr = yl[b][0][lane], ji = yl[b][1][lane];
#pragma unroll
      for (int a = 0; a < B; ++a) {
        const double mab = m[b * B + a];
        tr[a] += mab * jr;
        ti[a] += mab * ji;
      }
    }
#pragma unroll
    for (int a = 0; a < B; ++a) q += yl[a0 + a][0][lane] * tr[a] + yl[a0 + a][1][lane] * ti[a];
  }
  return 2.0 * q;
}

}  // namespace heget
