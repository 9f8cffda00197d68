// C ABI of the matrix-element library: process lookup, device state, launches.
#include "heget.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <sstream>
#include <string>

#include "heget_kernel_common.hpp"

extern const heget_proc_desc* const heget_registry[];
extern const int heget_registry_len;

struct heget_process {
  const heget_proc_desc* desc;
  int precision;
  int device;
  double* colour_table_dev;
};

namespace {

std::string normalise(const char* spec) {
  std::istringstream in(spec);
  std::string tok, out;
  while (in >> tok) {
    if (!out.empty()) out += ' ';
    out += tok;
  }
  return out;
}

const heget_proc_desc* find(const std::string& spec) {
  for (int i = 0; i < heget_registry_len; ++i)
    if (spec == heget_registry[i]->spec) return heget_registry[i];
  return nullptr;
}

}  // namespace

extern "C" {

heget_status heget_create_process(const char* spec, heget_precision precision, heget_process_t* out) {
  if (!spec || !out) return HEGET_E_INVALID_ARG;
  *out = nullptr;
  if (precision != HEGET_FP64 && precision != HEGET_MIXED) return HEGET_E_INVALID_ARG;
  const heget_proc_desc* d = find(normalise(spec));
  if (!d) return HEGET_E_UNSUPPORTED_PROCESS;
  heget_process* p = new (std::nothrow) heget_process{d, (int)precision, 0, nullptr};
  if (!p) return HEGET_E_OUT_OF_MEMORY;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return HEGET_E_DEVICE;
  }
  if (d->colour_table_len > 0) {
    const size_t bytes = sizeof(double) * (size_t)d->colour_table_len;
    if (hipMalloc(&p->colour_table_dev, bytes) != hipSuccess) {
      delete p;
      return HEGET_E_OUT_OF_MEMORY;
    }
    if (hipMemcpy(p->colour_table_dev, d->colour_table, bytes, hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(p->colour_table_dev);
      delete p;
      return HEGET_E_DEVICE;
    }
  }
  *out = p;
  return HEGET_OK;
}

heget_status heget_process_info(heget_process_t p, int* n_ext, int* n_diagrams, int* n_colours, int* n_helicities) {
  if (!p) return HEGET_E_INVALID_ARG;
  if (n_ext) *n_ext = p->desc->n_ext;
  if (n_diagrams) *n_diagrams = p->desc->n_diagrams;
  if (n_colours) *n_colours = p->desc->n_colours;
  if (n_helicities) *n_helicities = p->desc->n_helicities;
  return HEGET_OK;
}

heget_status heget_matrix_elements(heget_process_t p, const double* momenta, int64_t n_events, double alpha_s,
                                   double* me2, void* stream) {
  if (!p) return HEGET_E_INVALID_ARG;
  if (n_events < 0 || n_events > (int64_t(1) << 36)) return HEGET_E_INVALID_ARG;
  if (!(alpha_s > 0.0) || !std::isfinite(alpha_s)) return HEGET_E_INVALID_ARG;
  if (n_events == 0) return HEGET_OK;
  if (!momenta || !me2) return HEGET_E_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(momenta) & 15u) != 0) return HEGET_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HEGET_E_DEVICE;
  if (dev != p->device) return HEGET_E_INVALID_ARG;
  const double g2 = 4.0 * M_PI * alpha_s;
  // 2: configurations with leg 0 at helicity -1 equal their all-flipped partners;
  // 1/4: initial spin average; g^(2(n-2)): couplings left out of the kernels.
  const double scale = 2.0 * 0.25 * std::pow(g2, p->desc->n_ext - 2);
  hipError_t e = p->desc->launch(p->precision, momenta, n_events, me2, p->colour_table_dev, scale,
                                 reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;
}

heget_status heget_color_matrix(heget_process_t p, int* n_colours, int64_t* num, int64_t* den, double* values) {
  if (!p || !n_colours) return HEGET_E_INVALID_ARG;
  const int k = p->desc->n_colours;
  *n_colours = k;
  for (int i = 0; i < k * k; ++i) {
    if (num) num[i] = p->desc->colour_num[i];
    if (den) den[i] = p->desc->colour_den[i];
    if (values) values[i] = (double)p->desc->colour_num[i] / (double)p->desc->colour_den[i];
  }
  return HEGET_OK;
}

heget_status heget_process_flops(heget_process_t p, int64_t* flops_per_event) {
  if (!p || !flops_per_event) return HEGET_E_INVALID_ARG;
  *flops_per_event = p->desc->flops_per_event;
  return HEGET_OK;
}

void heget_destroy_process(heget_process_t p) {
  if (!p) return;
  if (p->colour_table_dev) hipFree(p->colour_table_dev);
  delete p;
}

const char* heget_status_string(heget_status s) {
  switch (s) {
    case HEGET_OK: return "ok";
    case HEGET_E_INVALID_ARG: return "invalid argument";
    case HEGET_E_UNSUPPORTED_PROCESS: return "unsupported process";
    case HEGET_E_OUT_OF_MEMORY: return "out of device memory";
    case HEGET_E_DEVICE: return "HIP device error";
  }
  return "unknown status";
}

int heget_num_processes(void) { return heget_registry_len; }

const char* heget_process_spec(int index) {
  if (index < 0 || index >= heget_registry_len) return nullptr;
  return heget_registry[index]->spec;
}

}  // extern "C"
