// Compact U(1) gauge sector (Sec. 5.3): placeholder entry points until the
// U(1) kernels land.
#include "common.hpp"
#include "internal.hpp"

namespace cl {

int u1_step(lattice*, int64_t) {
  set_error("U(1) model not built yet");
  return LAT_EINVAL;
}
int u1_energies(lattice*) {
  set_error("U(1) model not built yet");
  return LAT_EINVAL;
}
int u1_init_gauge(lattice*, double) {
  set_error("U(1) model not built yet");
  return LAT_EINVAL;
}

}  // namespace cl
