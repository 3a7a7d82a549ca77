// qbx_layer_potential_noalloc: the plain forward of qbx_layer_potential with
// its scratch arrays in one file-scope device array instead of a caller
// workspace, for callers that cannot allocate device memory (code under graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array is sized QBX_STATIC_SCRATCH_BYTES.  Every GPU the library runs on
// holds its own copy, at its own address, from the module's load until the
// process ends.  Its device address is looked up once per device with that
// device current, and only that address is handed to kernels: in host code the
// array's name is a host-side stand-in, not a device pointer.
//
// Every array the forward reads from the scratch is written earlier in the same
// call (tables, source grid, centers and J tables, then one partial sum per
// (source split, center)), so nothing needs clearing between calls.  All calls
// on one GPU share its copy: calls that overlap on one GPU (two streams, two
// threads) race and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qbx.h"
#include "qbx_internal.h"

static __device__ __align__(256) unsigned char scratch[QBX_STATIC_SCRATCH_BYTES];

namespace qbx {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// device address of this device's copy of `scratch`, looked up on first use
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(QBX_EDEVICE, "device %d is beyond the %d devices the static scratch serves", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_fail(e, "hipGetSymbolAddress of the static scratch");
    if (!p) return fail(QBX_EDEVICE, "hipGetSymbolAddress gave a NULL static scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QBX_OK;
}

}  // namespace
}  // namespace qbx

using namespace qbx;

extern "C" int qbx_layer_potential_noalloc(const qbx_geometry* g, const double* density,
                                           double k, int p, double r, int oversample, int side,
                                           int kind, double* out, hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!out) return fail(QBX_EINVAL, "out is NULL");
  const Layout L = make_forward_layout(d);
  if (L.total > (size_t)QBX_STATIC_SCRATCH_BYTES)
    return fail(QBX_EWORKSPACE,
                "this forward needs %zu bytes of scratch; the static scratch holds %zu",
                L.total, (size_t)QBX_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return run_forward(d, L, g->nodes, density, out, ws, stream, /*timed=*/false);
}
