// lbem_util_kernels.hpp -- small kernels used by several translation units
// (media packing and validation, zero fill, deterministic partial sums).
// Defined static so that every translation unit launches its own copy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbem.h"
#include "lbem_common.hpp"

namespace lbem {

// Fill a float array with a value, or copy src into it.
static __global__ void fill_or_copy(float *dst, const float *src, float value, uint32_t N) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < N) dst[i] = src ? src[i] : value;
}

static __global__ void zero_bytes(uint32_t *dst, size_t nwords) {
    const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < nwords) dst[i] = 0u;
}

// counts[0] non-finite, [1] non-positive eps/mu or negative sigma,
// [2] eps mu < 1, [3] HV sigma / (3 eps) >= 2
static __global__ void validate_media(const float *eps, const float *mu, const float *sig, uint32_t N, int model,
                               int32_t *counts) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    const float e = eps[i], m = mu[i], s = sig[i];
    if (!isfinite(e) || !isfinite(m) || !isfinite(s)) {
        atomicAdd(&counts[0], 1);
        return;
    }
    if (!(e > 0.f) || !(m > 0.f) || s < 0.f) atomicAdd(&counts[1], 1);
    else if (double(e) * double(m) < 1.0 - 1e-6) atomicAdd(&counts[2], 1);
    if (model == LBEM_HV && s / (3.0f * e) >= 2.0f) atomicAdd(&counts[3], 1);
}

// Deterministic sum of n partials into out[0] (one block).
static __global__ __launch_bounds__(kBlock) void sum_partials(const double *part, uint32_t n, double *out) {
    __shared__ double sm[4];
    double s = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) s += part[i];
    s = block_sum(s, sm);
    if (threadIdx.x == 0) out[0] = s;
}


}  // namespace lbem
