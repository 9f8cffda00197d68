// Device-side phase space, jet cuts and the event-weight sum of one integration step.
//
// The paper's program structure (section 3.2) turns host-drawn random numbers into
// momenta on the GPU (step 4), evaluates the colour-summed |M|^2 there (steps 4-5)
// and sums event weights into the cross section (step 7).  Here:
//   rambo_kernel   massless RAMBO (Kleiss, Stirling, Ellis 1986): n isotropic vectors
//                  with energy density q0 exp(-q0), boosted and scaled to (sqrt s, 0);
//                  the weight is the constant massless n-body phase-space volume;
//   cuts           pT > pT_min, |eta| < eta_max and pairwise Delta R > Delta R_min
//                  on every final parton (section 2.2, eqs. cuts; Delta R replaces the
//                  relative-pT cut);
//   weight_kernel  f = (hbar c)^2 * PS weight * |M|^2 * pass / (2 s S) with S the
//                  identical-final-parton factor, plus per-block sums of f and f^2;
//   sum_kernel     one block adding the block partials in index order (deterministic).
// One thread per event; the work is tiny next to the |M|^2 kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>

#include "heget.h"
#include "heget_internal.hpp"

namespace {

constexpr int kThreads = 256;
constexpr double kGeV2pb = 0.3893793721e9;   // (hbar c)^2 in pb GeV^2

__host__ __device__ double rambo_volume(int n, double s) {
  // (2 pi)^(4 - 3n) (pi / 2)^(n - 1) s^(n - 2) / ((n - 1)! (n - 2)!)
  double v = 1.0;
  for (int i = 0; i < n - 1; ++i) v *= 0.5 * M_PI;
  for (int i = 0; i < n - 2; ++i) v *= s;
  for (int i = 2; i <= n - 1; ++i) v /= (double)i;
  for (int i = 2; i <= n - 2; ++i) v /= (double)i;
  const double tp = 2.0 * M_PI;
  for (int i = 0; i < 3 * n - 4; ++i) v /= tp;
  return v;
}

template <int NF>
__global__ __launch_bounds__(kThreads) void rambo_kernel(int64_t nev, const double* __restrict__ sqrt_s,
                                                         const double* __restrict__ uni, double* __restrict__ mom,
                                                         double* __restrict__ psw) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= nev) return;
  const double rs = sqrt_s[e];
  const double* u = uni + e * NF * 4;
  double q[NF][4];
  double Q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const double c = 2.0 * u[4 * i + 0] - 1.0;
    const double st = sqrt(fmax(0.0, 1.0 - c * c));
    double sp, cp;
    sincospi(2.0 * u[4 * i + 1], &sp, &cp);
    const double e0 = -log(u[4 * i + 2] * u[4 * i + 3] + 1e-300);
    q[i][0] = e0;
    q[i][1] = e0 * st * cp;
    q[i][2] = e0 * st * sp;
    q[i][3] = e0 * c;
#pragma unroll
    for (int j = 0; j < 4; ++j) Q[j] += q[i][j];
  }
  const double m = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  const double b[3] = {-Q[1] / m, -Q[2] / m, -Q[3] / m};
  const double g = Q[0] / m;
  const double a = 1.0 / (1.0 + g);
  const double x = rs / m;
  double* out = mom + e * (NF + 2) * 4;
  const double h = 0.5 * rs;
  out[0] = h; out[1] = 0.0; out[2] = 0.0; out[3] = h;
  out[4] = h; out[5] = 0.0; out[6] = 0.0; out[7] = -h;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const double bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
    double* o = out + 8 + 4 * i;
    o[0] = x * (g * q[i][0] + bq);
#pragma unroll
    for (int j = 0; j < 3; ++j) o[1 + j] = x * (q[i][1 + j] + b[j] * q[i][0] + a * bq * b[j]);
  }
  if (psw) psw[e] = rambo_volume(NF, rs * rs);
}

__device__ bool passes(const double* fin, int nf, double pt_min, double eta_max, double dr_min) {
  double eta[8], phi[8];
  for (int i = 0; i < nf; ++i) {
    const double* p = fin + 4 * i;
    const double pt = sqrt(p[1] * p[1] + p[2] * p[2]);
    const double pa = sqrt(pt * pt + p[3] * p[3]);
    if (!(pt > pt_min)) return false;
    eta[i] = 0.5 * log((pa + p[3]) / fmax(pa - p[3], 1e-300));
    if (!(fabs(eta[i]) < eta_max)) return false;
    phi[i] = atan2(p[2], p[1]);
  }
  if (dr_min > 0.0) {
    for (int i = 0; i < nf; ++i)
      for (int j = i + 1; j < nf; ++j) {
        double dphi = fabs(phi[i] - phi[j]);
        if (dphi > M_PI) dphi = 2.0 * M_PI - dphi;
        const double deta = eta[i] - eta[j];
        if (!(sqrt(deta * deta + dphi * dphi) > dr_min)) return false;
      }
  }
  return true;
}

__global__ __launch_bounds__(kThreads) void cuts_kernel(int n_ext, int64_t nev, const double* __restrict__ mom,
                                                        double pt_min, double eta_max, double dr_min,
                                                        uint8_t* __restrict__ pass) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= nev) return;
  pass[e] = passes(mom + e * n_ext * 4 + 8, n_ext - 2, pt_min, eta_max, dr_min) ? 1 : 0;
}

// Block sums of f and f^2 with a fixed-shape tree, so results do not depend on timing.
__device__ void block_sum2(double a, double b, double* out) {
  __shared__ double sa[kThreads], sb[kThreads];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
}

__global__ __launch_bounds__(kThreads) void weight_kernel(int n_ext, int64_t nev, const double* __restrict__ mom,
                                                          const double* __restrict__ me2, double factor,
                                                          double pt_min, double eta_max, double dr_min,
                                                          double* __restrict__ weight, double* __restrict__ part) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double f = 0.0;
  if (e < nev) {
    const double* p = mom + e * n_ext * 4;
    const double s = 4.0 * p[0] * p[4];   // (p_a + p_b)^2 for back-to-back massless beams
    if (passes(p + 8, n_ext - 2, pt_min, eta_max, dr_min))
      f = factor * rambo_volume(n_ext - 2, s) * me2[e] / (2.0 * s);
    weight[e] = f;
  }
  block_sum2(f, f * f, part + 2 * (int64_t)blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void sum_kernel(int64_t nblocks, const double* __restrict__ part,
                                                       double* __restrict__ sums) {
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nblocks; i += kThreads) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  block_sum2(a, b, sums);
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// Work space of heget_integrate_step_noalloc: the weight kernel's per-block partial sums (f, f^2),
// one pair per 256 events, in a fixed device array instead of stream-ordered allocations.  Every
// block of a launch writes its own pair, so nothing has to be cleared between calls.
constexpr int64_t kScratchBlocks = int64_t(1) << 17;                  // 2 MiB: up to 2^25 events
constexpr int64_t kNoallocMaxEvents = kScratchBlocks * kThreads;

}  // namespace

static __device__ __align__(256) double scratch[2 * kScratchBlocks];

namespace {

// Device address of `scratch` on each device (host code may not use the symbol's name itself).
std::mutex g_scratch_mutex;
std::map<int, double*> g_scratch_ptr;

hipError_t scratch_for_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    it = g_scratch_ptr.emplace(dev, static_cast<double*>(ptr)).first;
  }
  *out = it->second;
  return hipSuccess;
}

bool valid_cuts(const heget_cuts* c) {
  return c && std::isfinite(c->pt_min) && std::isfinite(c->eta_max) && std::isfinite(c->delta_r_min) &&
         c->eta_max > 0.0;
}

hipError_t launch_rambo(int nf, int64_t n, const double* rs, const double* u, double* mom, double* psw,
                        hipStream_t s) {
  const dim3 g(blocks(n)), b(kThreads);
  switch (nf) {
    case 2: hipLaunchKernelGGL(rambo_kernel<2>, g, b, 0, s, n, rs, u, mom, psw); break;
    case 3: hipLaunchKernelGGL(rambo_kernel<3>, g, b, 0, s, n, rs, u, mom, psw); break;
    case 4: hipLaunchKernelGGL(rambo_kernel<4>, g, b, 0, s, n, rs, u, mom, psw); break;
    case 5: hipLaunchKernelGGL(rambo_kernel<5>, g, b, 0, s, n, rs, u, mom, psw); break;
    case 6: hipLaunchKernelGGL(rambo_kernel<6>, g, b, 0, s, n, rs, u, mom, psw); break;
    case 7: hipLaunchKernelGGL(rambo_kernel<7>, g, b, 0, s, n, rs, u, mom, psw); break;
    case 8: hipLaunchKernelGGL(rambo_kernel<8>, g, b, 0, s, n, rs, u, mom, psw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

heget_status heget_rambo(int n_final, int64_t n_events, const double* sqrt_s, const double* uniforms,
                         double* momenta, double* ps_weight, void* stream) {
  if (n_final < 2 || n_final > 8 || n_events < 0 || n_events > (int64_t(1) << 36)) return HEGET_E_INVALID_ARG;
  if (n_events == 0) return HEGET_OK;
  if (!sqrt_s || !uniforms || !momenta) return HEGET_E_INVALID_ARG;
  const hipError_t e = launch_rambo(n_final, n_events, sqrt_s, uniforms, momenta, ps_weight,
                                    reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;
}

heget_status heget_apply_cuts(int n_ext, int64_t n_events, const double* momenta, const heget_cuts* cuts,
                              uint8_t* pass, void* stream) {
  if (n_ext < 4 || n_ext > 10 || n_events < 0 || n_events > (int64_t(1) << 36) || !valid_cuts(cuts))
    return HEGET_E_INVALID_ARG;
  if (n_events == 0) return HEGET_OK;
  if (!momenta || !pass) return HEGET_E_INVALID_ARG;
  hipLaunchKernelGGL(cuts_kernel, dim3(blocks(n_events)), dim3(kThreads), 0, reinterpret_cast<hipStream_t>(stream),
                     n_ext, n_events, momenta, cuts->pt_min, cuts->eta_max, cuts->delta_r_min, pass);
  return hipGetLastError() == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;
}

}  // extern "C"

namespace {

// Both integration-step entry points: with part == nullptr the block partials are taken from and
// returned to the stream-ordered pool, otherwise they go to part (at least 2 * blocks(n) doubles)
// and nothing is allocated (the sampled-helicity mode then runs without the chirality sort).
heget_status integrate_step(heget_process_t p, int64_t n_events, const double* sqrt_s, const double* uniforms,
                            const int32_t* helicity, double alpha_s, const heget_cuts* cuts, double* momenta,
                            double* me2, double* weight, double* sums, void* stream, double* part) {
  int n_ext = 0;
  if (!p || heget_process_info(p, &n_ext, nullptr, nullptr, nullptr) != HEGET_OK) return HEGET_E_INVALID_ARG;
  if (n_events <= 0 || n_events > (int64_t(1) << 36) || !valid_cuts(cuts)) return HEGET_E_INVALID_ARG;
  if (!sqrt_s || !uniforms || !momenta || !me2 || !weight || !sums) return HEGET_E_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(momenta) & 15u) != 0) return HEGET_E_INVALID_ARG;
  if (!(alpha_s > 0.0) || !std::isfinite(alpha_s)) return HEGET_E_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (launch_rambo(n_ext - 2, n_events, sqrt_s, uniforms, momenta, nullptr, s) != hipSuccess) return HEGET_E_DEVICE;
  const bool own = part == nullptr;
  heget_status st = helicity ? heget_detail_matrix_elements_helicity(p, momenta, helicity, n_events, alpha_s, me2,
                                                                     stream, own)
                             : heget_matrix_elements(p, momenta, n_events, alpha_s, me2, stream);
  if (st != HEGET_OK) return st;
  // identical final partons: 1 / prod(k!) over the species of the final state
  double factor = kGeV2pb / heget_detail_final_symmetry(p);
  if (helicity) factor *= (double)(int64_t(1) << n_ext);   // one sampled configuration stands for 2^n
  const int64_t nb = blocks(n_events);
  if (own && hipMallocAsync(&part, sizeof(double) * 2 * nb, s) != hipSuccess) return HEGET_E_OUT_OF_MEMORY;
  hipLaunchKernelGGL(weight_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, n_ext, n_events, momenta, me2, factor,
                     cuts->pt_min, cuts->eta_max, cuts->delta_r_min, weight, part);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kThreads), 0, s, nb, part, sums);
  const hipError_t e = hipGetLastError();
  if (own) (void)hipFreeAsync(part, s);
  return e == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;
}

}  // namespace

extern "C" {

heget_status heget_integrate_step(heget_process_t p, int64_t n_events, const double* sqrt_s, const double* uniforms,
                                  const int32_t* helicity, double alpha_s, const heget_cuts* cuts, double* momenta,
                                  double* me2, double* weight, double* sums, void* stream) {
  return integrate_step(p, n_events, sqrt_s, uniforms, helicity, alpha_s, cuts, momenta, me2, weight, sums, stream,
                        nullptr);
}

heget_status heget_integrate_step_noalloc(heget_process_t p, int64_t n_events, const double* sqrt_s,
                                          const double* uniforms, const int32_t* helicity, double alpha_s,
                                          const heget_cuts* cuts, double* momenta, double* me2, double* weight,
                                          double* sums, void* stream) {
  if (n_events > kNoallocMaxEvents) return HEGET_E_INVALID_ARG;
  double* part = nullptr;
  if (n_events > 0 && scratch_for_current_device(&part) != hipSuccess) return HEGET_E_DEVICE;
  return integrate_step(p, n_events, sqrt_s, uniforms, helicity, alpha_s, cuts, momenta, me2, weight, sums, stream,
                        part);
}

}  // extern "C"
