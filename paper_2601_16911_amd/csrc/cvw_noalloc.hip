// Allocation-free variant of cvw_residual, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc): the operation's workspace is a fixed per-device array of
// this library instead of a caller buffer.
//
// The array lives as long as the process on every device the entry point has
// run on.  Its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and kept; the array's name is
// never used as a device address in host code.  Every call on a device shares
// that device's array: calls that overlap on one device (other streams, other
// host threads) race and must not be issued.
#include <mutex>

#include "cvw_internal.h"

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;   // 16 MiB per device

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// zero the status words at the head of the workspace (a kernel, so that the
// call holds no memset node when captured into a graph)
__global__ void clear_status_words(uint32_t* __restrict__ w) {
  if (threadIdx.x < 64) w[threadIdx.x] = 0u;
}

// the device address of `scratch` on device `dev` (current); nullptr on error
void* scratch_of(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" cvw_status cvw_residual_noalloc(const cvw_mesh* m, const cvw_params* prm, const void* u, void* R,
                                           void* gamma_out, void* stream) {
  if (!m || !prm) { cvw::set_error("null argument"); return CVW_EINVAL; }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    cvw::set_error("no current device"); return CVW_EDEVICE;
  }
  if (dev != m->device) { cvw::set_error("the current device is not the mesh's device"); return CVW_EINVAL; }
  const size_t need = cvw_workspace_bytes(m, prm, 0);
  if (need == 0 || need > NOALLOC_SCRATCH_BYTES) {
    cvw::set_error("this mesh and operation need " + std::to_string(need) +
                   " bytes of workspace; the allocation-free residual holds 16 MiB (16777216 bytes) per device");
    return CVW_EINVAL;
  }
  void* ws = scratch_of(dev);
  if (!ws) { cvw::set_error("hipGetSymbolAddress of the scratch array failed"); return CVW_EDEVICE; }
  auto s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(clear_status_words, dim3(1), dim3(64), 0, s, static_cast<uint32_t*>(ws));
  if (hipGetLastError() != hipSuccess) { cvw::set_error("kernel launch failed"); return CVW_EDEVICE; }
  return cvw_residual(m, prm, u, R, gamma_out, ws, NOALLOC_SCRATCH_BYTES, stream);
}
