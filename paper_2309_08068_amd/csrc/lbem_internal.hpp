// lbem_internal.hpp -- host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/lbem.h"
#include "lbem_common.hpp"

namespace lbem {

// Byte offsets of the regions of a lattice workspace.
struct WsLayout {
    size_t pop, rec, eps, mu, sig, en_part, det_part, src_blk, src_cell, src_J0, src_tp, prb_blk, prb_cell, prb_slot, flx_cell,
        flags;
    size_t det_cap;  // detector partial slots
    size_t total;
};

WsLayout layout(const lbem_desc *d);

// Threads per block of the row form of the step kernel (one block per x-row):
// nx itself for 128, 256, 384, 512, else the next of 128, 256, 384, 512 when
// the row fills at least 3/4 of it (threads past nx idle); 0 when the lattice
// uses the generic form.  Measured on MI355X: rows that fill 3/4 of their
// block gain 2-18 points of the HBM peak over the generic form (100, 120, 192,
// 250, 300, 320, 500 cells), once their stores finish the row's last write
// piece (see RowIO).
inline uint32_t row_block(const lbem_desc *d) {
    const uint32_t nx = uint32_t(d->nx);
    if (nx == 128 || nx == 256 || nx == 384 || nx == 512) return nx;
    if (nx < 96 || nx > 512) return 0u;
    const uint32_t rb = nx <= 128 ? 128u : nx <= 256 ? 256u : nx <= 384 ? 384u : 512u;
    return 4 * nx >= 3 * rb ? rb : 0u;
}

// Equilibrium-shifted storage formats keep two planes of 16-byte per-cell
// records (the step at time t reads plane (t + 1) & 1 and writes plane t & 1).
// Populations per cell of a model, 0 for an unknown model.
inline int model_pops(int32_t model) {
    return model == LBEM_MM ? 50 : model == LBEM_HV ? 36 : model == LBEM_MM_DIFF ? 24 : 0;
}
inline bool shifted(int32_t storage) { return storage == LBEM_BF16_SHIFTED || storage == LBEM_F16_SHIFTED; }
// Population layout (see PopLayout): row-form lattices use chunks of a power
// of two of x-rows with at most kChunkBytes per population plane (measured on
// MI355X: 32 KB beat 16 KB, 64 KB and larger chunks and the plain [Q][N]
// layout, which was up to 15 % slower on large lattices); a lattice that fits
// in one chunk, and every generic-form lattice, is a single chunk of N cells.
constexpr uint32_t kChunkBytes = 32768;
inline PopLayout pop_layout(const lbem_desc *d) {
    const uint32_t Q = uint32_t(model_pops(d->model));
    const uint32_t s = d->storage == LBEM_F32 ? 4u : 2u;
    const uint32_t cells = kChunkBytes / s;
    const uint64_t rows = uint64_t(d->ny) * d->nz;
    // row-form rows are a power of two of cells apart (the padding cells are
    // never touched).  Measured on MI355X: rows that start mid-line cost every
    // one of their Q plane accesses an extra partial cache line, and rows of
    // 1.5 KB (384 cells) ran at 71-75 % of the HBM peak against 79 % with a
    // 2 KB pitch (and 32 KB plane chunks instead of 24 KB)
    uint32_t pitch = uint32_t(d->nx);
    if (row_block(d))
        while (pitch & (pitch - 1u)) pitch += pitch & (~pitch + 1u);  // next power of two
    PopLayout L{uint32_t(d->nx), 31u, uint32_t(rows * pitch), 0, pitch};
    if (row_block(d)) {
        uint32_t sh = 0;
        while ((uint64_t(2) << sh) * pitch <= cells) ++sh;
        if ((uint64_t(1) << sh) < rows) {
            L.rshift = sh;
            L.C = (1u << sh) * pitch;
        }
    }
    L.QC = uint64_t(Q) * L.C;
    return L;
}
inline uint64_t pop_elems(const lbem_desc *d) {
    const PopLayout L = pop_layout(d);
    const uint64_t rows = uint64_t(d->ny) * d->nz;
    const uint64_t nchunks = L.rshift == 31 ? 1 : (rows + (uint64_t(1) << L.rshift) - 1) >> L.rshift;
    return nchunks * L.QC;
}
inline size_t pop_bytes(const lbem_desc *d) { return size_t(pop_elems(d)) * (d->storage == LBEM_F32 ? 4 : 2); }
constexpr size_t kRecBytes = 16;
// Bytes of one saved state: the populations, and for the shifted formats the
// record plane the next step reads.
inline size_t state_bytes(const lbem_desc *d) {
    return pop_bytes(d) + (shifted(d->storage) ? size_t(d->nx) * d->ny * d->nz * kRecBytes : 0);
}


// Record a message for lbem_last_error and return st.
lbem_status fail(lbem_status st, const char *fmt, ...);
lbem_status hip_check(hipError_t e, const char *what);

// 2 pi n / period + phase with whole periods removed in double precision.

// Arguments of one launch of the 3-D step kernel.
struct StepArgs {
    void *pop;
    PopLayout pl;
    const float *eps, *mu, *sig;
    uint32_t nx, ny, nz, N;
    float scale, inv_scale;
    // soft current sources: per-block ranges into a cell-sorted list; source k
    // carries J0[3k..3k+2] sin(2 pi t / tp[2k] + tp[2k+1]) at time level src_t
    const int32_t *src_blk, *src_cell;
    const float *src_J0;
    const double *src_tp;
    double src_t;
    // hard plane source
    int32_t plane_z;
    float Eimp[3], Bimp[3];
    // probes: per-block ranges, cell, output slot; prb_row = this step's row
    const int32_t *prb_blk, *prb_cell, *prb_slot;
    double *prb_row;
    // detector plane
    int32_t det_z;
    uint32_t det_b0, det_b1;
    double *det_part;
    // energy partials (null: not this step)
    double *en_part;
    // if set, E of the collided state is written here ([3][N] floats)
    float *E_out;
    // shifted storage: the two record planes (uint4 [N] each), else null
    void *rec[2];
    // > 0: blocks in the grouped XCD order with groups of this many blocks
    // (see xcd_block); 0: hardware order
    uint32_t xcd_group;
};


}  // namespace lbem

struct lbem_lattice {
    lbem_desc d;
    int Q;
    size_t sbytes;
    uint32_t N;
    uint32_t bu;       // cells per step-kernel block and per table unit (nx in row form, else 256)
    uint32_t nblocks;  // step-kernel blocks = table units, ceil(N / bu)
    uint32_t nobs;     // blocks of the 256-thread observation kernels
    float scale, inv_scale;
    int device;  // the GPU current at lbem_create
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    lbem::WsLayout L;
    lbem::PopLayout pl;
    // sources (host copy of the list, in the order given)
    int32_t nsrc;
    std::vector<int32_t> src_cells;
    std::vector<float> src_J0;
    std::vector<double> src_tp;
    int32_t plane_z;
    float pE0[3], pB0[3];
    double plane_period;
    // probes
    int32_t nprobe;
    int64_t prb_cap, prb_t0;
    double *prb_series;
    // energy-flux monitor
    int32_t flx_n;
    int64_t flx_t0, flx_t1;
    double *flx_max;
    // detector; det_acc: caller buffer that receives the accumulated sum after
    // every lbem_step call (lbem_set_detector_plane), or null
    int32_t det_z;
    uint32_t det_b0, det_b1;
    double *det_acc;
    // energy series
    int32_t en_every;
    int64_t en_cap, en_t0;
    double *en_series;
    int64_t t;
    // launch tuning of the step kernel per parity: address form, blocks per CU
    // cap, and the dynamic LDS that implements the cap
    int32_t tune_form[2], tune_cap[2];
    size_t tune_pad[2];
    // adjoint session (lbem_adjoint_forward)
    void *adj_ws;
    int64_t adj_t0, adj_nsteps;
    int32_t adj_K, adj_keep, adj_det;
    // launch tuning of the adjoint row kernel per parity (chosen on the first
    // reverse pass): form (0 LDS, early addresses; 1 LDS, late; 2 direct),
    // blocks-per-CU cap and its dynamic LDS
    int32_t adj_tuned, adj_form[2], adj_cap[2];
    size_t adj_pad[2];
};


namespace lbem {
// Amplitude weight sin(2 pi t / period + phase) of a soft source (host side:
// the hard plane source), with the whole periods removed from t / period first.
inline double source_weight(double t, double period, double phase) {
    const double r = t / period;
    return sin(2.0 * M_PI * (r - floor(r)) + phase);
}

// The same weight in the step kernels, without a library sine (whose inlined
// code would raise every kernel's register allocation): the argument is
// reduced in FP64 to u = (t / period + phase / 2 pi) mod 1 in [-1/2, 1/2],
// then x = 2 pi u is folded into [-pi/2, pi/2] with sin(x) = sin(+-pi - x), and
// sin x is the odd Taylor series to x^15 in FP32 (truncation below 1e-9 there;
// the result is accurate to FP32 rounding, far inside the 1e-5 parity bar).
__device__ inline float source_weight_dev(double t, double period, double phase) {
    double u = t / period + phase * (0.5 / M_PI);
    u -= rint(u);
    float x = float(u) * 6.28318530717958647692f;
    const float hp = 1.57079632679489661923f, pi = 3.14159265358979323846f;
    if (x > hp) x = pi - x;
    else if (x < -hp) x = -pi - x;
    const float x2 = x * x;
    // x (1 - x^2/3! (1 - x^2/(4.5) (1 - ... ))) written as Horner in x^2
    float p = 1.0f / 1307674368000.0f;            // 1/15!
    p = p * -x2 + 1.0f / 6227020800.0f;           // 1/13!
    p = p * -x2 + 1.0f / 39916800.0f;             // 1/11!
    p = p * -x2 + 1.0f / 362880.0f;               // 1/9!
    p = p * -x2 + 1.0f / 5040.0f;                 // 1/7!
    p = p * -x2 + 1.0f / 120.0f;                  // 1/5!
    p = p * -x2 + 1.0f / 6.0f;                    // 1/3!
    p = p * -x2 + 1.0f;
    return x * p;
}
// Step-kernel arguments for the lattice's current configuration (no
// observation or frame output set).
StepArgs base_step_args(lbem_lattice *lat);
// Dynamic LDS that caps the resident blocks of `kernel` per compute unit at
// cap (0: no cap), given its static LDS.
size_t lds_pad_for(const void *kernel, int cap);
// Workgroups per x-row of the step kernel chosen for this parity (1 unless
// the row is split, tuning form 3).
uint32_t step_segments(const lbem_lattice *lat, int odd);
// Launch one step kernel of the lattice's model and storage.
void dispatch_step(const lbem_lattice *lat, const StepArgs &a, int odd);
// lbem_step with every observation; if frames is set, E of the state collided
// by step s is also written to frames + s * 3 N.
lbem_status step_impl(lbem_lattice *lat, int64_t nsteps, float *frames);
}  // namespace lbem
