// Forward synthesis without any allocation: the scratch that iris_rt_forward
// takes from the caller's workspace (the temperature tables of the cell
// setup and the erfc pieces of the thin modes) comes instead from a
// file-scope device array, one copy per GPU, for callers that cannot allocate
// device memory (code under graph capture, tight serving loops).

#include <hip/hip_runtime.h>

#include <mutex>

#include "host_common.h"

using namespace iris::host;

namespace {

// Largest scratch a call may need: the forward without checkpoints, reading
// the fields in place, uses the table and erfc regions of the workspace
// (about 104 KiB); 128 KiB leaves room for their 256-byte alignment.
constexpr size_t kScratchBytes = 128 * 1024;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each GPU, looked up once per device with that
// device current. In host code `scratch` names a host-side stand-in, never the
// device memory: only these pointers are passed to kernels.
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

iris_status scratch_on_current_device(void** ptr) {
  int dev = -1;
  int e = (int)hipGetDevice(&dev);
  if (e) return hip_status(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(IRIS_E_UNSUPPORTED, "device %d beyond the %d the static scratch serves", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e) return hip_status(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(IRIS_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = p;
  }
  *ptr = g_scratch[dev];
  return IRIS_OK;
}

}  // namespace

extern "C" {

size_t iris_rt_forward_static_max_bytes(void) { return kScratchBytes; }

iris_status iris_rt_forward_static(const iris_fields* fields, const iris_channels* channels,
                                   const iris_line* line, const iris_outputs* out, void* stream) {
  clear_error();
  Geo g;
  iris_status s;
  if ((s = check_fields(fields, &g)) != IRIS_OK) return s;
  if ((s = check_channels(channels)) != IRIS_OK) return s;
  const size_t need = ws_layout(fields, g, march_channels(channels).n_chan, 0).total;
  if (need > kScratchBytes)
    return fail(IRIS_E_WORKSPACE,
                "this forward needs %zu bytes of scratch, above the static scratch's %zu "
                "(a sightline-major copy of the fields is not available here)",
                need, kScratchBytes);
  void* ws = nullptr;
  if ((s = scratch_on_current_device(&ws)) != IRIS_OK) return s;
  return forward_impl(fields, channels, line, out, 0, ws, kScratchBytes, stream, 0);
}

}  // extern "C"
