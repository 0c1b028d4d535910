// lattice_energies_noalloc: the observables of a lattice with the per-block
// FP64 partial sums of their passes kept in a file-scope device array instead
// of the workspace, for callers that cannot allocate device memory.  The
// passes, their kernels and their order are those of lattice_energies, so the
// results are the same to the bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace cl {

constexpr size_t kScratchBytes = (size_t)4 << 20;  // 4 MiB per device, held until the process ends

// One copy per device.  In host code `scratch` names a host-side stand-in, not
// device memory: kernels and copies get the address noalloc_setup() obtained.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;  // device address of `scratch`, per device

// Record the device address of `scratch` for the current device (once).
int noalloc_setup() {
  int dev = 0;
  CL_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (g_scratch_ptr[(size_t)dev]) return LAT_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return LAT_EHIP;
  }
  g_scratch_ptr[(size_t)dev] = ptr;
  return LAT_OK;
}

static void* scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (size_t)dev < g_scratch_ptr.size() ? g_scratch_ptr[(size_t)dev] : nullptr;
}

// Bytes of per-block partial records the observation passes of h write.
// Scalar: one observation pass on its fixed tile, 5 nf + 3 FP64 sums per
// tile.  U(1): the Gauss residual (4 per 256 sites),
// then the pass on the lattice's tile (11 per tile).  SU(2) x U(1): the Gauss
// residuals and the pass, at most 16 per 256 sites.
static size_t energy_partial_bytes(const lattice* h) {
  const size_t N = (size_t)h->p.N, V = N * N * N;
  if (is_su2(h->p)) return V / 256 * 16 * sizeof(double);
  if (is_u1(h->p)) {
    const Tiling& t = h->tile;
    const size_t tiles = (N / (size_t)t.tz) * (N / (size_t)(t.by * t.ry)) * (N / (size_t)t.xc);
    return std::max(V / 256 * 4, tiles * 11) * sizeof(double);
  }
  return (size_t)scalar_obs_blocks(h->p.N) * (size_t)(5 * h->p.nf + 3) * sizeof(double);
}

}  // namespace cl

using namespace cl;

extern "C" int lattice_energies_noalloc(lattice_t* h, lattice_obs* out) {
  if (!h || !out) { set_error("NULL argument"); return LAT_EINVAL; }
  const size_t need = energy_partial_bytes(h);
  if (need > kScratchBytes) {
    set_error("lattice_energies_noalloc: the partial sums need " + std::to_string(need) +
              " bytes, above the 4 MiB static scratch (use lattice_energies)");
    return LAT_ENOMEM;
  }
  int rc = noalloc_setup();  // a no-op after lattice_init on this device
  if (rc) return rc;
  void* ptr = scratch_ptr();
  if (!ptr) { set_error("lattice_energies_noalloc: no scratch address for this device"); return LAT_EHIP; }
  // Every block writes its whole record before the finish reads it, so
  // nothing in the scratch has to start at zero.
  double* const saved = h->partials;
  h->partials = static_cast<double*>(ptr);
  rc = is_u1(h->p) ? u1_energies(h) : is_su2(h->p) ? su2_energies(h) : scalar_energies(h);
  h->partials = saved;
  if (rc) return rc;
  DevState d;
  CL_HIP(hipMemcpyAsync(&d, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
  CL_HIP(hipStreamSynchronize(h->stream));
  *out = d.obs;
  out->step = h->step;
  out->staggered = h->staggered;
  if (d.nonfinite) { set_error("non-finite volume average"); return LAT_ENONFINITE; }
  return LAT_OK;
}
