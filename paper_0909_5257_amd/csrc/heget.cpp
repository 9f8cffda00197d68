// C ABI of the matrix-element library: process lookup, device state, launches.
#include "heget.h"
#include "heget_internal.hpp"

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "heget_kernel_common.hpp"

extern const heget_proc_desc* const heget_registry[];
extern const int heget_registry_len;

struct heget_process {
  const heget_proc_desc* desc;
  int precision;
  int device;
  double* colour_table_dev;
  int* pattern_dev;      // helicity bit pattern -> chirality pattern (processes with several)
  uint64_t serial;       // unique per handle ever created (cached graphs are keyed by it)
};

namespace {

std::atomic<uint64_t> g_next_serial{1};
void forget_graphs_of(uint64_t serial);

std::string normalise(const char* spec) {
  std::istringstream in(spec);
  std::string tok, out;
  while (in >> tok) {
    if (!out.empty()) out += ' ';
    out += tok;
  }
  return out;
}

// Sort key of each event of the sampled-helicity mode: its chirality pattern, or n_patterns for a
// structural zero or an out-of-range pattern (those do no work and are sorted last).
__global__ void pattern_keys(const int32_t* __restrict__ hel, int n, int n_ext, const int* __restrict__ table,
                             int n_patterns, int* __restrict__ keys, int* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int h = hel[i];
  int k = n_patterns;
  if (h >= 0 && h < (1 << n_ext) && table[h] >= 0) k = table[h];
  keys[i] = k;
  idx[i] = i;
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
  heget_process* p = new (std::nothrow) heget_process{d, (int)precision, 0, nullptr, nullptr, g_next_serial++};
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
      (void)hipFree(p->colour_table_dev);
      delete p;
      return HEGET_E_DEVICE;
    }
  }
  if (d->n_patterns > 1) {
    const size_t bytes = sizeof(int) * ((size_t)1 << d->n_ext);
    if (hipMalloc(&p->pattern_dev, bytes) != hipSuccess) {
      heget_destroy_process(p);
      return HEGET_E_OUT_OF_MEMORY;
    }
    if (hipMemcpy(p->pattern_dev, d->helicity_pattern, bytes, hipMemcpyHostToDevice) != hipSuccess) {
      heget_destroy_process(p);
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
  hipError_t e = p->desc->launch(p->precision, momenta, nullptr, nullptr, n_events, me2, p->colour_table_dev,
                                 scale, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;
}

heget_status heget_matrix_elements_helicity(heget_process_t p, const double* momenta, const int32_t* helicity,
                                            int64_t n_events, double alpha_s, double* me2, void* stream) {
  return heget_detail_matrix_elements_helicity(p, momenta, helicity, n_events, alpha_s, me2, stream, true);
}

}  // extern "C"

heget_status heget_detail_matrix_elements_helicity(heget_process_t p, const double* momenta, const int32_t* helicity,
                                                   int64_t n_events, double alpha_s, double* me2, void* stream,
                                                   bool allow_sort) {
  if (!p) return HEGET_E_INVALID_ARG;
  if (n_events < 0 || n_events > (int64_t(1) << 36)) return HEGET_E_INVALID_ARG;
  if (!(alpha_s > 0.0) || !std::isfinite(alpha_s)) return HEGET_E_INVALID_ARG;
  if (n_events == 0) return HEGET_OK;
  if (!momenta || !helicity || !me2) return HEGET_E_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(momenta) & 15u) != 0) return HEGET_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HEGET_E_DEVICE;
  if (dev != p->device) return HEGET_E_INVALID_ARG;
  const double g2 = 4.0 * M_PI * alpha_s;
  // one term of the helicity sum: 1/4 initial spin average and the couplings, no flip factor
  const double scale = 0.25 * std::pow(g2, p->desc->n_ext - 2);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!allow_sort || p->pattern_dev == nullptr || n_events >= (int64_t(1) << 31) ||
      n_events > p->desc->max_launch_events) {
    hipError_t e = p->desc->launch(p->precision, momenta, helicity, nullptr, n_events, me2, p->colour_table_dev,
                                   scale, s);
    return e == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;
  }
  // several chirality patterns: order the events by pattern (stable radix sort of the pattern
  // keys) so that a workgroup's 64 events share one pattern and run one pass instead of all
  const int n = (int)n_events;
  int *keys = nullptr, *keys_out = nullptr, *idx = nullptr, *perm = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  int bits = 1;
  while ((1 << bits) <= p->desc->n_patterns) ++bits;
  heget_status st = HEGET_OK;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys, keys_out, idx, perm, n, 0, bits, s) !=
      hipSuccess)
    return HEGET_E_DEVICE;
  const size_t nb = sizeof(int) * (size_t)n;
  if (hipMallocAsync(&keys, nb, s) != hipSuccess || hipMallocAsync(&keys_out, nb, s) != hipSuccess ||
      hipMallocAsync(&idx, nb, s) != hipSuccess || hipMallocAsync(&perm, nb, s) != hipSuccess ||
      hipMallocAsync(&temp, temp_bytes, s) != hipSuccess) {
    st = HEGET_E_OUT_OF_MEMORY;
  } else {
    hipLaunchKernelGGL(pattern_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, helicity, n,
                       p->desc->n_ext, p->pattern_dev, p->desc->n_patterns, keys, idx);
    if (hipGetLastError() != hipSuccess ||
        hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_out, idx, perm, n, 0, bits, s) != hipSuccess ||
        p->desc->launch(p->precision, momenta, helicity, perm, n_events, me2, p->colour_table_dev, scale, s) !=
            hipSuccess)
      st = HEGET_E_DEVICE;
  }
  for (void* b : {(void*)keys, (void*)keys_out, (void*)idx, (void*)perm, temp})
    if (b) (void)hipFreeAsync(b, s);
  return st;
}

extern "C" {

heget_status heget_matrix_elements_hook(heget_process_t p, const double* momenta, int64_t n_events, double alpha_s,
                                        int gauge_leg, double* me2, double* jamp, void* stream) {
  if (!p) return HEGET_E_INVALID_ARG;
  if (!p->desc->launch_hook) return HEGET_E_UNSUPPORTED_PROCESS;
  if (n_events < 0 || n_events > (int64_t(1) << 36)) return HEGET_E_INVALID_ARG;
  if (!(alpha_s > 0.0) || !std::isfinite(alpha_s)) return HEGET_E_INVALID_ARG;
  if (gauge_leg < -1 || gauge_leg >= p->desc->n_ext) return HEGET_E_INVALID_ARG;
  if (gauge_leg >= 0) {
    // only gluon legs carry a polarisation vector
    std::istringstream in(p->desc->spec);
    std::string tok;
    int leg = 0;
    bool gluon = false;
    while (in >> tok) {
      if (tok == ">") continue;
      if (leg++ == gauge_leg) gluon = tok == "g";
    }
    if (!gluon) return HEGET_E_INVALID_ARG;
  }
  if (n_events == 0) return HEGET_OK;
  if (!momenta || !me2) return HEGET_E_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(momenta) & 15u) != 0) return HEGET_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HEGET_E_DEVICE;
  if (dev != p->device) return HEGET_E_INVALID_ARG;
  const double scale = 2.0 * 0.25 * std::pow(4.0 * M_PI * alpha_s, p->desc->n_ext - 2);
  hipError_t e = p->desc->launch_hook(p->precision, momenta, n_events, me2, p->colour_table_dev, scale, gauge_leg,
                                      jamp, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;
}

heget_status heget_colour_reduction(heget_process_t p, int* k_reduced, int* n_slots, int64_t* m_num, int64_t* m_den,
                                    int64_t* w_num, int64_t* w_den, int32_t* slot_helicity) {
  if (!p || !k_reduced || !n_slots) return HEGET_E_INVALID_ARG;
  const heget_proc_desc* d = p->desc;
  *k_reduced = d->k_reduced;
  *n_slots = d->n_slots;
  const int64_t nm = (int64_t)d->k_reduced * d->n_colours, nw = (int64_t)d->k_reduced * d->k_reduced;
  for (int64_t i = 0; i < nm; ++i) {
    if (m_num) m_num[i] = d->red_num[i];
    if (m_den) m_den[i] = d->red_den[i];
  }
  for (int64_t i = 0; i < nw; ++i) {
    if (w_num) w_num[i] = d->w_num[i];
    if (w_den) w_den[i] = d->w_den[i];
  }
  if (slot_helicity)
    for (int i = 0; i < d->n_slots; ++i) slot_helicity[i] = d->slot_helicity[i];
  return HEGET_OK;
}

}  // extern "C"

namespace {

constexpr int kBatchStreams = 4;
constexpr size_t kGraphCacheMax = 32;

struct DevicePool {
  hipStream_t streams[kBatchStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t done[kBatchStreams] = {};
  hipStream_t capture = nullptr;
  bool ready = false;
};

struct GraphEntry {
  hipGraphExec_t exec;
  uint64_t last_use;
  std::vector<uint64_t> serials;   // handles the captured launches use
};

std::mutex g_batch_mutex;
std::map<int, DevicePool> g_pools;
std::map<std::string, GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;

hipError_t pool_for(int dev, DevicePool** out) {
  DevicePool& p = g_pools[dev];
  if (!p.ready) {
    for (int i = 0; i < kBatchStreams; ++i) {
      hipError_t e = hipStreamCreateWithFlags(&p.streams[i], hipStreamNonBlocking);
      if (e != hipSuccess) return e;
      e = hipEventCreateWithFlags(&p.done[i], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    e = hipStreamCreateWithFlags(&p.capture, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    p.ready = true;
  }
  *out = &p;
  return hipSuccess;
}

double item_scale(const heget_proc_desc* d, double alpha_s) {
  return 2.0 * 0.25 * std::pow(4.0 * M_PI * alpha_s, d->n_ext - 2);
}

// Fork from `origin`, launch the items longest-first on the pool streams, join back.
hipError_t enqueue_batch(DevicePool* pool, const heget_batch_item* items, int n, double alpha_s,
                         hipStream_t origin) {
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cost = [&](int i) {
    return (double)items[i].process->desc->algo_flops_per_event * (double)items[i].n_events;
  };
  std::sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  double load[kBatchStreams] = {0.0};
  bool used[kBatchStreams] = {false};
  hipError_t e = hipEventRecord(pool->fork, origin);
  if (e != hipSuccess) return e;
  for (int s = 0; s < kBatchStreams; ++s) {
    e = hipStreamWaitEvent(pool->streams[s], pool->fork, 0);
    if (e != hipSuccess) return e;
  }
  for (int i : order) {
    if (items[i].n_events == 0) continue;
    int s = (int)(std::min_element(load, load + kBatchStreams) - load);
    load[s] += cost(i);
    used[s] = true;
    const heget_process* p = items[i].process;
    e = p->desc->launch(p->precision, items[i].momenta, nullptr, nullptr, items[i].n_events, items[i].me2,
                        p->colour_table_dev,
                        item_scale(p->desc, alpha_s), pool->streams[s]);
    if (e != hipSuccess) return e;
  }
  for (int s = 0; s < kBatchStreams; ++s) {
    e = hipEventRecord(pool->done[s], pool->streams[s]);
    if (e != hipSuccess) return e;
    e = hipStreamWaitEvent(origin, pool->done[s], 0);
    if (e != hipSuccess) return e;
  }
  (void)used;
  return hipSuccess;
}

// Key of a captured batch: device, alpha_s and per item the handle's serial (never reused, unlike
// the handle's address), the buffers and the size.
std::string batch_key(const heget_batch_item* items, int n, double alpha_s, int dev) {
  std::string key(reinterpret_cast<const char*>(&dev), sizeof(dev));
  key.append(reinterpret_cast<const char*>(&alpha_s), sizeof(alpha_s));
  for (int i = 0; i < n; ++i) {
    const uint64_t serial = items[i].process->serial;
    key.append(reinterpret_cast<const char*>(&serial), sizeof(serial));
    key.append(reinterpret_cast<const char*>(&items[i].momenta), sizeof(items[i].momenta));
    key.append(reinterpret_cast<const char*>(&items[i].n_events), sizeof(items[i].n_events));
    key.append(reinterpret_cast<const char*>(&items[i].me2), sizeof(items[i].me2));
  }
  return key;
}

// Drop every cached graph that launches a kernel of the handle with this serial.
void forget_graphs_of(uint64_t serial) {
  std::lock_guard<std::mutex> lock(g_batch_mutex);
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    const auto& ser = it->second.serials;
    if (std::find(ser.begin(), ser.end(), serial) != ser.end()) {
      (void)hipGraphExecDestroy(it->second.exec);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace

extern "C" {

heget_status heget_matrix_elements_batch(const heget_batch_item* items, int n_items, double alpha_s,
                                         int use_graph, void* stream) {
  if (n_items < 0 || (n_items > 0 && !items)) return HEGET_E_INVALID_ARG;
  if (!(alpha_s > 0.0) || !std::isfinite(alpha_s)) return HEGET_E_INVALID_ARG;
  int dev = -1;
  if (n_items == 0) return HEGET_OK;
  if (hipGetDevice(&dev) != hipSuccess) return HEGET_E_DEVICE;
  for (int i = 0; i < n_items; ++i) {
    const heget_batch_item& it = items[i];
    if (!it.process || it.n_events < 0 || it.n_events > (int64_t(1) << 36)) return HEGET_E_INVALID_ARG;
    if (it.process->device != dev) return HEGET_E_INVALID_ARG;
    if (it.n_events > 0 && (!it.momenta || !it.me2)) return HEGET_E_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(it.momenta) & 15u) != 0) return HEGET_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_batch_mutex);
  DevicePool* pool = nullptr;
  if (pool_for(dev, &pool) != hipSuccess) return HEGET_E_DEVICE;
  hipStream_t origin = reinterpret_cast<hipStream_t>(stream);
  if (!use_graph) return enqueue_batch(pool, items, n_items, alpha_s, origin) == hipSuccess ? HEGET_OK : HEGET_E_DEVICE;

  const std::string key = batch_key(items, n_items, alpha_s, dev);
  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    // capture on a library stream (the caller's may be the legacy default stream)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(pool->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return HEGET_E_DEVICE;
    hipError_t e = enqueue_batch(pool, items, n_items, alpha_s, pool->capture);
    hipError_t e2 = hipStreamEndCapture(pool->capture, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return HEGET_E_DEVICE;
    }
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return HEGET_E_DEVICE;
    if (g_graphs.size() >= kGraphCacheMax) {
      auto victim = std::min_element(g_graphs.begin(), g_graphs.end(), [](const auto& a, const auto& b) {
        return a.second.last_use < b.second.last_use;
      });
      (void)hipGraphExecDestroy(victim->second.exec);
      g_graphs.erase(victim);
    }
    std::vector<uint64_t> serials;
    for (int i = 0; i < n_items; ++i) serials.push_back(items[i].process->serial);
    it = g_graphs.emplace(key, GraphEntry{exec, 0, std::move(serials)}).first;
  }
  it->second.last_use = ++g_graph_clock;
  // order the replay after and before the caller's stream
  if (hipEventRecord(pool->fork, origin) != hipSuccess) return HEGET_E_DEVICE;
  if (hipStreamWaitEvent(pool->capture, pool->fork, 0) != hipSuccess) return HEGET_E_DEVICE;
  if (hipGraphLaunch(it->second.exec, pool->capture) != hipSuccess) return HEGET_E_DEVICE;
  if (hipEventRecord(pool->done[0], pool->capture) != hipSuccess) return HEGET_E_DEVICE;
  if (hipStreamWaitEvent(origin, pool->done[0], 0) != hipSuccess) return HEGET_E_DEVICE;
  return HEGET_OK;
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
  *flops_per_event = p->desc->algo_flops_per_event;
  return HEGET_OK;
}

void heget_destroy_process(heget_process_t p) {
  if (!p) return;
  forget_graphs_of(p->serial);
  if (p->colour_table_dev) (void)hipFree(p->colour_table_dev);
  if (p->pattern_dev) (void)hipFree(p->pattern_dev);
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

double heget_detail_final_symmetry(heget_process_t p) {
  // prod over final-state species of (multiplicity)!
  std::istringstream in(p->desc->spec);
  std::string tok;
  bool final_state = false;
  std::map<std::string, int> count;
  while (in >> tok) {
    if (tok == ">") {
      final_state = true;
      continue;
    }
    if (final_state) ++count[tok];
  }
  double f = 1.0;
  for (const auto& kv : count)
    for (int i = 2; i <= kv.second; ++i) f *= (double)i;
  return f;
}
