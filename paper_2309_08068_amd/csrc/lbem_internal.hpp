// lbem_internal.hpp -- host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lbem.h"

namespace lbem {

// Byte offsets of the regions of a lattice workspace.
struct WsLayout {
    size_t pop, eps, mu, sig, en_part, det_part, src_blk, src_cell, src_J0, prb_blk, prb_cell, prb_slot, flags;
    size_t det_cap;  // detector partial slots
    size_t total;
};

WsLayout layout(const lbem_desc *d);

// Record a message for lbem_last_error and return st.
lbem_status fail(lbem_status st, const char *fmt, ...);
lbem_status hip_check(hipError_t e, const char *what);

// 2 pi n / period + phase with whole periods removed in double precision.
double two_pi_frac(double n, double period, double phase);

}  // namespace lbem
