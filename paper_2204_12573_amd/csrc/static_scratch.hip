// Allocation-free virial: the variant of flare_virial whose FP64 task sums live in a
// fixed, file-scope device array instead of state memory the library grows on demand.
//
// The array is a module-scope __device__ variable, so every GPU the library runs on holds
// its own copy (1 MiB, until the process ends). In host code its name is only a stand-in
// for that symbol, never a device address: the address is looked up once per device, with
// that device current, through hipGetSymbolAddress and kept in a per-device table, and only
// that pointer is passed to kernels.
//
// Every call on one GPU shares that GPU's copy and leaves the last call's task sums in it.
// The kernels write every task sum before the per-cell pass reads it, so nothing has to
// start at zero; calls that overlap on one GPU (two streams at once) race on the array.
#include <mutex>

#include "state.h"

namespace {

constexpr size_t SCRATCH_DOUBLES = 131072;           // 1 MiB
constexpr size_t MAX_TASKS = SCRATCH_DOUBLES / 9;     // 14,563 reduction tasks of 9 sums
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch` (dev must be current).
int scratch_for_device(int dev, double** out) {
  if (dev < 0 || dev >= MAX_DEVICES) {
    flare::set_error("device index beyond the static scratch table");
    return FLARE_E_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      flare::set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return FLARE_E_HIP;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FLARE_OK;
}

}  // namespace

extern "C" int flare_virial_noalloc(flare_state* s, double* virial_struct) {
  if (!s || !virial_struct) {
    flare::set_error("null pointer");
    return FLARE_E_ARG;
  }
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) {
    flare::set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return FLARE_E_HIP;
  }
  if (cur != s->device) {
    flare::set_error("the state's device must be the current device");
    return FLARE_E_ARG;
  }
  if (!s->have_desc || s->w_gen != s->pos_gen) {
    flare::set_error("flare_virial_noalloc needs forces (flare_energy_forces or flare_forces) for the current positions");
    return FLARE_E_STALE;
  }
  if (s->tasks.size() > MAX_TASKS) {
    flare::set_error("flare_virial_noalloc: " + std::to_string(s->tasks.size()) + " reduction tasks, the static " +
                     "scratch holds " + std::to_string(MAX_TASKS));
    return FLARE_E_CAPACITY;
  }
  double* red = nullptr;
  const int rc = scratch_for_device(cur, &red);
  if (rc != FLARE_OK) return rc;
  flare::virial_cells(s, virial_struct, red);    // no stage timer: its events are created on demand
  e = hipGetLastError();
  if (e != hipSuccess) {
    flare::set_error(std::string("virial kernels: ") + hipGetErrorString(e));
    return FLARE_E_HIP;
  }
  return FLARE_OK;
}
