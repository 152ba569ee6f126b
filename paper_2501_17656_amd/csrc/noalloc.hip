// The fixed device scratch region of the solve that allocates nothing.
//
// A file-scope device array holds the solve's vectors for callers that
// cannot allocate device memory.  Host code never passes the array's name to
// a kernel or a copy: the name is a host-side stand-in, not a device
// address.  The device address is looked up once per device, with that
// device current, and every use goes through it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdexcept>
#include <string>

#include "h2_build.h"

namespace h2mg {

namespace {

static __device__ __align__(256) unsigned char scratch[H2MG_SOLVE_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
void* scratch_addr[MAX_DEVICES] = {};

}  // namespace

void* solve_scratch(size_t* bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) throw std::runtime_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) throw std::runtime_error("device index out of range for the solve scratch");
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw std::runtime_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    scratch_addr[dev] = p;
  }
  *bytes = H2MG_SOLVE_SCRATCH_BYTES;
  return scratch_addr[dev];
}

}  // namespace h2mg
