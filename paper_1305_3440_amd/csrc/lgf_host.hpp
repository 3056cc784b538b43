// lgf_host.hpp -- host-side helpers shared by the C-ABI translation units:
// error reporting, argument checks, lattice geometry.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lgf.h"
#include "lgf_device.hpp"

namespace lgf {

// record a message for lgf_last_error() and return st
lgf_status fail(lgf_status st, const char *fmt, ...);

bool valid_format(int f);
bool valid_dims(const int dims[4]);
Geom make_geom(const int dims[4]);
double elapsed_ms(hipEvent_t a, hipEvent_t b);

}  // namespace lgf

#define LGF_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::lgf::fail(LGF_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                               __FILE__, __LINE__);                                            \
    } while (0)

#define LGF_TRY(expr)                                                                          \
    do {                                                                                       \
        lgf_status s_ = (expr);                                                                \
        if (s_ != LGF_OK) return s_;                                                           \
    } while (0)
