// msg_internal.hpp -- functions shared between the host scheduler
// (msg_host.cpp) and the no-allocation entry point (noalloc.hip).
#pragma once
#include <stddef.h>

#include "../../include/msg.h"

namespace msg {

// the body of msg_sample_field: its device staging in `staging` (cap bytes),
// or allocated on the stream for the call when staging is null
msg_status sample_field_impl(msg_handle h, const msg_field_spec* spec, const msg_batch_desc* batch,
                             const double* d_xi, double* d_kx, double* d_ky, float* d_kx32, float* d_ky32,
                             msg_stream stream, void* staging, size_t cap);
// the HIP device a handle is bound to
int handle_device(msg_handle h);
// record `text` as this thread's msg_last_error() and return st
msg_status report(msg_status st, const char* text);
// with `device` current: the device address of that device's no-allocation
// scratch, looked up once per device (noalloc.hip)
msg_status noalloc_setup(int device);

}  // namespace msg
