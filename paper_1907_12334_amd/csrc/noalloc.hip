// noalloc.hip -- msg_sample_field_noalloc: the field synthesis with its device
// staging in a static array instead of memory allocated per call, for callers
// that cannot allocate (code under HIP graph capture, serving loops that
// forbid allocation).
//
// The array `scratch` below lives in every device's copy of this code object.
// In host code its name is a host-side stand-in, not a device address: the
// address of a device's copy is looked up once per device, with that device
// current, when a handle is created (noalloc_setup, from msg_create), and
// only that address is ever passed to kernels or copies.  All calls on one
// device share its array and it keeps the last call's contents; the staging
// written by a call is complete before its kernels read it (same stream), and
// nothing in it needs to start at zero.  Calls that overlap on one device
// (two host threads, or two streams in flight) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/msg.h"
#include "msg_internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;   // 32 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

msg_status msg::noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return report(MSG_ERR_ARG, "device index outside 0..63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return MSG_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return report(MSG_ERR_HIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    g_ptr[device] = p;
    return MSG_OK;
}

extern "C" msg_status msg_sample_field_noalloc(msg_handle h, const msg_field_spec* spec, const msg_batch_desc* batch,
                                              const double* d_xi, double* d_kx, double* d_ky, float* d_kx32,
                                              float* d_ky32, msg_stream stream)
{
    if (!h) return msg::report(MSG_ERR_ARG, "handle is NULL");
    const int dev = msg::handle_device(h);
    void* p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (dev >= 0 && dev < kMaxDevices) p = g_ptr[dev];
    }
    if (!p) return msg::report(MSG_ERR_HIP, "the no-allocation scratch of the handle's device is not set up");
    return msg::sample_field_impl(h, spec, batch, d_xi, d_kx, d_ky, d_kx32, d_ky32, stream, p, kScratchBytes);
}
