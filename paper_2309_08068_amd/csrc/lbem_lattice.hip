// lbem_lattice.hip -- kernels and C ABI of the 3-D lattice (include/lbem.h).
//
// One kernel launch performs one complete time step of Appendix B for every
// cell: gather the populations (in-place AA streaming), collide (Section II or
// III), impose hard sources, scatter, and -- when requested for this step --
// record probes, the detector-plane |E|^2 and per-block energy partials in
// FP64.  One thread owns one cell; cells are numbered x fastest, and a
// workgroup owns one x-row (or a 128-cell piece of one) whose population
// planes are contiguous runs of the layout chunk the row lies in (PopLayout),
// or, in the generic form, a run of 256 cells of the [Q][N] layout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbem.h"
#include "lbem_common.hpp"
#include "lbem_internal.hpp"
#include "lbem_util_kernels.hpp"

using namespace lbem;

// ============================================================== kernels

// Generic form: one thread per cell, neighbours addressed directly, blocks of
// 256 cells (any lattice shape; such lattices are a single layout chunk).
template <class M, int ODD, class ST>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a) {
    constexpr int NW = kBlock / 64;
    __shared__ double sm_en[NW], sm_det[NW];
    const uint32_t blk = a.xcd_group ? xcd_block(blockIdx.x, gridDim.x, a.xcd_group) : blockIdx.x;
    const uint32_t c = blk * kBlock + threadIdx.x;
    const bool live = c < a.N;
    const uint32_t cc = live ? c : a.N - 1;
    const uint32_t nxy = a.nx * a.ny;
    const uint32_t z = cc / nxy, rem = cc - z * nxy, y = rem / a.nx, x = rem - y * a.nx;
    const Nbr nb = make_nbr(cc, x, y, z, a.nx, a.ny, a.nz);
    const size_t N = a.N;
    const size_t P = a.pl.C;  // population plane stride: generic lattices are a single chunk
    auto *pop = static_cast<typename ST::T *>(a.pop);

    float f[M::Q];
    if (live) gather<M, ODD, ST>(pop, P, nb, f, a.inv_scale);
    else
        for (int q = 0; q < M::Q; ++q) f[q] = 0.f;
    if constexpr (ST::kShift)
        if (live)
            unshift<M>(f, static_cast<const u32x4 *>(a.rec[ODD ? 0 : 1]),
                       [&](int dx, int dy, int dz) { return nb.at(dx, dy, dz); });

    CellMedia m{a.eps[cc], a.mu[cc], a.sig[cc]};
    float Js[3] = {0.f, 0.f, 0.f};
    if (a.src_blk) {
        const int s0 = a.src_blk[blk], s1 = a.src_blk[blk + 1];
        for (int k = s0; k < s1; ++k)
            if (a.src_cell[k] == int32_t(c)) {
                const float w = source_weight_dev(a.src_t, a.src_tp[2 * k], a.src_tp[2 * k + 1]);
                Js[0] = a.src_J0[3 * k] * w;
                Js[1] = a.src_J0[3 * k + 1] * w;
                Js[2] = a.src_J0[3 * k + 2] * w;
            }
    }
    CellFields o;
    Cell<M>::collide(f, m, Js, o);
    const bool plane = int32_t(z) == a.plane_z;
    if (plane) Cell<M>::equilibrium(f, m, a.Eimp, a.Bimp);
    if constexpr (ST::kShift)
        shift_out<M>(f, plane ? a.Eimp : o.E, plane ? a.Bimp : o.B, m.eps_r, m.mu_r,
                     static_cast<u32x4 *>(a.rec[ODD ? 1 : 0]), c, live);
    if (live) {
        // store addresses formed after the collision (see late_addresses)
        Nbr nb2 = nb;
        auto *pop2 = pop;
        late_addresses(nb2, pop2, f[0]);
        scatter<M, ODD, ST>(pop2, P, nb2, f, a.scale);
    }

    // ---- observation of the state this step collided
    if (a.E_out && live) {  // frames are read back once, much later: non-temporal
        __builtin_nontemporal_store(o.E[0], a.E_out + c);
        __builtin_nontemporal_store(o.E[1], a.E_out + N + c);
        __builtin_nontemporal_store(o.E[2], a.E_out + 2 * N + c);
    }
    if (a.prb_blk) {
        const int p0 = a.prb_blk[blk], p1 = a.prb_blk[blk + 1];
        for (int k = p0; k < p1; ++k)
            if (a.prb_cell[k] == int32_t(c)) {
                double *o6 = a.prb_row + 6 * a.prb_slot[k];
                o6[0] = o.E[0]; o6[1] = o.E[1]; o6[2] = o.E[2];
                o6[3] = o.B[0]; o6[4] = o.B[1]; o6[5] = o.B[2];
            }
    }
    if (a.det_part && blk >= a.det_b0 && blk <= a.det_b1) {
        const double e2 = (live && int32_t(z) == a.det_z)
                              ? double(o.E[0]) * o.E[0] + double(o.E[1]) * o.E[1] + double(o.E[2]) * o.E[2]
                              : 0.0;
        const double s = block_sum<NW>(e2, sm_det);
        if (threadIdx.x == 0) a.det_part[(blk - a.det_b0) * kSegMax] += s;
    }
    if (a.en_part) {
        const double u = live ? 0.5 * (double(o.E[0]) * o.D[0] + double(o.E[1]) * o.D[1] + double(o.E[2]) * o.D[2] +
                                       double(o.B[0]) * o.H[0] + double(o.B[1]) * o.H[1] + double(o.B[2]) * o.H[2])
                              : 0.0;
        const double s = block_sum<NW>(u, sm_en);
        if (threadIdx.x == 0) a.en_part[blk] = s;
    }
}

// Row form of the step for lattices with x extent nx <= RB: TB threads per
// block, RB / TB blocks per x-row (y and z are uniform per block; threads
// past nx idle), see RowIO.  Same arithmetic as step_kernel, bit for bit.
// LATE = 1 forms the store addresses after the collision (see late_addresses);
// DIRECT = 1 addresses the x-shifted cells in HBM instead of through LDS (a
// split row, TB < RB, needs it).  Which variant is faster depends on model,
// storage, parity and row length, so all exist and the launch tuning picks one.
template <class M, int ODD, class ST, int RB, int LATE, int DIRECT, int TB = RB>
__global__ __launch_bounds__(TB) void row_step_kernel(StepArgs a) {
    static_assert(RB % TB == 0 && (TB == RB || DIRECT), "a split row needs direct addressing");
    constexpr int NW = TB / 64, SEG = RB / TB;
    using T = typename ST::T;
    __shared__ T sh[(ODD && !DIRECT) ? n_xshift<M>() : 1][RB];
    __shared__ double sm_en[NW], sm_det[NW];
    const uint32_t blk = a.xcd_group ? xcd_block(blockIdx.x, gridDim.x, a.xcd_group) : blockIdx.x;
    const uint32_t row = blk / SEG, seg = blk % SEG;  // row = y + ny z
    const uint32_t x = seg * TB + threadIdx.x;
    const uint32_t z = row / a.ny;
    const bool live = x < a.nx;  // rows shorter than RB leave the last threads idle
    const uint32_t c = row * a.nx + (live ? x : 0u);
    const size_t N = a.N;
    RowIO<M, ST, RB> io(a.pop, a.pl, a.ny, a.nz, row, x);
    // shifted storage: the LDS forms of MM and the difference form exchange
    // the x-shifted records (RecX)
    using RX = RecX<M, RB>;
    constexpr bool XREC = ST::kShift && !DIRECT && RX::kUse;
    __shared__ float xs[XREC ? RX::kX * RX::P : 1][XREC ? RB : 1];
    float un[XREC ? RX::kN : 1][RX::P];
    if constexpr (XREC) RX::publish(io, static_cast<const u32x4 *>(a.rec[ODD ? 0 : 1]), xs, un);
    float f[M::Q];
    if (DIRECT) {
        io.template gather_direct<ODD>(f, a.inv_scale);
    } else if constexpr (XREC && ODD) {
        // the gather's first barrier orders the xs writes; read them in its read phase
        io.template gather<ODD>(f, sh, a.inv_scale, [&](float (&g)[M::Q]) { RX::collect(io, xs, un, g); });
    } else {
        io.template gather<ODD>(f, sh, a.inv_scale);
        if constexpr (XREC) {
            lds_phase_barrier();
            RX::collect(io, xs, un, f);
        }
    }
    if constexpr (ST::kShift && !XREC) {
        if (live)
            unshift<M>(f, static_cast<const u32x4 *>(a.rec[ODD ? 0 : 1]),
                       [&](int dx, int dy, int dz) { return io.cell(dx, dy, dz); });
    }

    CellMedia m{a.eps[c], a.mu[c], a.sig[c]};
    float Js[3] = {0.f, 0.f, 0.f};
    if (a.src_blk && live) {
        const int s0 = a.src_blk[row], s1 = a.src_blk[row + 1];
        for (int k = s0; k < s1; ++k)
            if (a.src_cell[k] == int32_t(c)) {
                const float w = source_weight_dev(a.src_t, a.src_tp[2 * k], a.src_tp[2 * k + 1]);
                Js[0] = a.src_J0[3 * k] * w;
                Js[1] = a.src_J0[3 * k + 1] * w;
                Js[2] = a.src_J0[3 * k + 2] * w;
            }
    }
    CellFields o;
    Cell<M>::collide(f, m, Js, o);
    const bool plane = int32_t(z) == a.plane_z;
    if (plane) Cell<M>::equilibrium(f, m, a.Eimp, a.Bimp);
    if constexpr (ST::kShift)
        shift_out<M>(f, plane ? a.Eimp : o.E, plane ? a.Bimp : o.B, m.eps_r, m.mu_r,
                     static_cast<u32x4 *>(a.rec[ODD ? 1 : 0]), c, live);

    if (LATE) io.late(f[0]);
    if (DIRECT) io.template scatter_direct<ODD>(f, a.scale);
    else io.template scatter<ODD>(f, sh, a.scale);

    // ---- observation of the state this step collided
    if (!live) {
        for (int k = 0; k < 3; ++k) o.E[k] = o.B[k] = o.D[k] = o.H[k] = 0.f;
    }
    if (a.E_out && live) {
        __builtin_nontemporal_store(o.E[0], a.E_out + c);
        __builtin_nontemporal_store(o.E[1], a.E_out + N + c);
        __builtin_nontemporal_store(o.E[2], a.E_out + 2 * N + c);
    }
    if (a.prb_blk && live) {
        const int p0 = a.prb_blk[row], p1 = a.prb_blk[row + 1];
        for (int k = p0; k < p1; ++k)
            if (a.prb_cell[k] == int32_t(c)) {
                double *o6 = a.prb_row + 6 * a.prb_slot[k];
                o6[0] = o.E[0]; o6[1] = o.E[1]; o6[2] = o.E[2];
                o6[3] = o.B[0]; o6[4] = o.B[1]; o6[5] = o.B[2];
            }
    }
    if (a.det_part && row >= a.det_b0 && row <= a.det_b1) {
        const double e2 = int32_t(z) == a.det_z
                              ? double(o.E[0]) * o.E[0] + double(o.E[1]) * o.E[1] + double(o.E[2]) * o.E[2]
                              : 0.0;
        const double s = block_sum<NW>(e2, sm_det);
        if (threadIdx.x == 0) a.det_part[(row - a.det_b0) * kSegMax + seg] += s;
    }
    if (a.en_part) {
        const double u = 0.5 * (double(o.E[0]) * o.D[0] + double(o.E[1]) * o.D[1] + double(o.E[2]) * o.D[2] +
                                double(o.B[0]) * o.H[0] + double(o.B[1]) * o.H[1] + double(o.B[2]) * o.H[2]);
        const double s = block_sum<NW>(u, sm_en);
        if (threadIdx.x == 0) a.en_part[row * SEG + seg] = s;
    }
}

struct ObsArgs {
    const void *pop;
    PopLayout pl;
    const float *eps, *mu, *sig;
    uint32_t nx, ny, nz, N;
    uint32_t bu;  // cells per source-table unit
    float inv_scale;
    const int32_t *src_blk, *src_cell;
    const float *src_J0;
    const double *src_tp;
    double src_t;
    float *E, *B, *D, *H;
    double *en_part;
    const void *rec;  // shifted storage: the record plane this state's reader uses
};

// Reported fields of cell cc of the current state.
template <class M, int ODD, class ST>
__device__ __forceinline__ void observe_cell(const ObsArgs &a, uint32_t cc, CellFields &o) {
    const uint32_t nxy = a.nx * a.ny;
    const uint32_t z = cc / nxy, rem = cc - z * nxy, y = rem / a.nx, x = rem - y * a.nx;
    const Nbr nb = make_nbr(cc, x, y, z, a.nx, a.ny, a.nz);
    float f[M::Q];
    gather_any<M, ODD, ST>(static_cast<const typename ST::T *>(a.pop), a.pl, nb, f, a.inv_scale);
    if constexpr (ST::kShift)
        unshift<M>(f, static_cast<const u32x4 *>(a.rec), [&](int dx, int dy, int dz) { return nb.at(dx, dy, dz); });
    CellMedia m{a.eps[cc], a.mu[cc], a.sig[cc]};
    float Js[3] = {0.f, 0.f, 0.f};
    if (a.src_blk) {
        const uint32_t u = cc / a.bu;
        const int s0 = a.src_blk[u], s1 = a.src_blk[u + 1];
        for (int k = s0; k < s1; ++k)
            if (a.src_cell[k] == int32_t(cc)) {
                const float w = source_weight_dev(a.src_t, a.src_tp[2 * k], a.src_tp[2 * k + 1]);
                Js[0] = a.src_J0[3 * k] * w;
                Js[1] = a.src_J0[3 * k + 1] * w;
                Js[2] = a.src_J0[3 * k + 2] * w;
            }
    }
    Cell<M>::collide(f, m, Js, o);
}

// Reported fields of the current state (no update).
template <class M, int ODD, class ST>
__global__ __launch_bounds__(kBlock) void observe_kernel(ObsArgs a) {
    __shared__ double sm_en[4];
    const uint32_t blk = blockIdx.x;
    const uint32_t c = blk * kBlock + threadIdx.x;
    const bool live = c < a.N;
    const size_t N = a.N;
    CellFields o;
    observe_cell<M, ODD, ST>(a, live ? c : a.N - 1, o);
    if (live) {
        for (int d = 0; d < 3; ++d) {
            if (a.E) a.E[d * N + c] = o.E[d];
            if (a.B) a.B[d * N + c] = o.B[d];
            if (a.D) a.D[d * N + c] = o.D[d];
            if (a.H) a.H[d * N + c] = o.H[d];
        }
    }
    if (a.en_part) {
        const double u = live ? 0.5 * (double(o.E[0]) * o.D[0] + double(o.E[1]) * o.D[1] + double(o.E[2]) * o.D[2] +
                                       double(o.B[0]) * o.H[0] + double(o.B[1]) * o.H[1] + double(o.B[2]) * o.H[2])
                              : 0.0;
        const double s = block_sum(u, sm_en);
        if (threadIdx.x == 0) a.en_part[blk] = s;
    }
}

// Energy-flux monitor: maxflux[k] = max(maxflux[k], |E x H|) of the reported
// fields in cells[k] (one thread per monitored cell).
template <class M, int ODD, class ST>
__global__ __launch_bounds__(kBlock) void flux_kernel(ObsArgs a, const int32_t *cells, uint32_t n, double *maxflux) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    CellFields o;
    observe_cell<M, ODD, ST>(a, uint32_t(cells[k]), o);
    const double Sx = double(o.E[1]) * o.H[2] - double(o.E[2]) * o.H[1];
    const double Sy = double(o.E[2]) * o.H[0] - double(o.E[0]) * o.H[2];
    const double Sz = double(o.E[0]) * o.H[1] - double(o.E[1]) * o.H[0];
    maxflux[k] = fmax(maxflux[k], sqrt(Sx * Sx + Sy * Sy + Sz * Sz));
}

// f := f_eq(E, B, J = 0) in natural layout.  Shifted storage: slot (q, c)
// holds f_q - phi_q(R_{c - v_q}) with the records of the same fields, which
// init_record_kernel has written to the plane the first step reads.
template <class M, class ST>
__global__ __launch_bounds__(kBlock) void init_kernel(void *pop, PopLayout pl, const float *eps, const float *mu,
                                                      const float *E, const float *B, uint32_t nx, uint32_t ny,
                                                      uint32_t nz, uint32_t N, float scale, const void *rec) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= N) return;
    CellMedia m{eps[c], mu[c], 0.f};
    const float e[3] = {E[c], E[size_t(N) + c], E[2 * size_t(N) + c]};
    const float b[3] = {B[c], B[size_t(N) + c], B[2 * size_t(N) + c]};
    float f[M::Q];
    Cell<M>::equilibrium(f, m, e, b);
    if constexpr (ST::kShift) {
        const uint32_t nxy = nx * ny;
        const uint32_t z = c / nxy, rem = c - z * nxy, y = rem / nx, x = rem - y * nx;
        const Nbr nb = make_nbr(c, x, y, z, nx, ny, nz);
        float g[M::Q];
        for (int q = 0; q < M::Q; ++q) g[q] = 0.f;
        unshift<M>(g, static_cast<const u32x4 *>(rec), [&](int dx, int dy, int dz) { return nb.at(dx, dy, dz); });
        for (int q = 0; q < M::Q; ++q) f[q] -= g[q];
    }
    auto *p = static_cast<typename ST::T *>(pop);
    const uint64_t i0 = pl.index(0, c);
#pragma unroll
    for (int q = 0; q < M::Q; ++q) ST::store(p + i0 + uint64_t(q) * pl.C, 0, f[q], scale);
}

__global__ __launch_bounds__(kBlock) void init_record_kernel(void *rec, const float *eps, const float *mu,
                                                             const float *E, const float *B, uint32_t N) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= N) return;
    const float e[3] = {E[c], E[size_t(N) + c], E[2 * size_t(N) + c]};
    const float b[3] = {B[c], B[size_t(N) + c], B[2 * size_t(N) + c]};
    Rec r;
    static_cast<u32x4 *>(rec)[c] = rec_pack(e, b, eps[c], 1.0f / mu[c], r);
}

// ============================================================== host side

namespace lbem {
thread_local char g_err[512] = "";

lbem_status fail(lbem_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

lbem_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return LBEM_OK;
    return fail(LBEM_EHIP, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace lbem

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool is_f16(int st) { return st == LBEM_F16 || st == LBEM_F16_SHIFTED; }

lbem_status check_desc(const lbem_desc *d) {
    if (!d) return fail(LBEM_EINVAL, "desc is NULL");
    if (model_pops(d->model) == 0) return fail(LBEM_EINVAL, "unknown model %d", d->model);
    if (d->storage < LBEM_F32 || d->storage > LBEM_F16_SHIFTED)
        return fail(LBEM_EINVAL, "unknown storage %d", d->storage);
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(LBEM_EINVAL, "lattice size must be >= 1 on every axis");
    if (d->reserved != 0) return fail(LBEM_EINVAL, "reserved field must be 0");
    const double n = double(d->nx) * d->ny * d->nz;
    if (n >= 2147483648.0) return fail(LBEM_EINVAL, "lattice has %.0f cells; the limit is 2^31 - 1", n);
    if (is_f16(d->storage) && d->storage_scale != 0.0) {
        int ex;
        const double m = std::frexp(d->storage_scale, &ex);
        if (!(d->storage_scale > 0.0) || m != 0.5) return fail(LBEM_EINVAL, "storage_scale must be a power of two");
    }
    return LBEM_OK;
}

size_t storage_bytes(int st) { return st == LBEM_F32 ? 4 : 2; }

}  // namespace

namespace lbem {
WsLayout layout(const lbem_desc *d) {
    WsLayout L;
    const size_t N = size_t(d->nx) * d->ny * d->nz;
    const size_t bu = row_block(d) ? size_t(d->nx) : kBlock;  // cells per block unit: a row, or kBlock cells
    const size_t nblocks = (N + bu - 1) / bu;
    const size_t nobs = (N + kBlock - 1) / kBlock;
    const size_t nxy = size_t(d->nx) * d->ny;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.pop = take(pop_bytes(d));
    L.rec = take(shifted(d->storage) ? 2 * N * kRecBytes : 0);
    L.eps = take(N * 4);
    L.mu = take(N * 4);
    L.sig = take(N * 4);
    L.en_part = take(std::max(nblocks * kSegMax, nobs) * 8);
    L.det_cap = nxy / bu + 2;
    L.det_part = take(L.det_cap * kSegMax * 8);
    L.src_blk = take((nblocks + 1) * 4);
    L.src_cell = take(size_t(LBEM_MAX_SOURCES) * 4);
    L.src_J0 = take(size_t(LBEM_MAX_SOURCES) * 12);
    L.src_tp = take(size_t(LBEM_MAX_SOURCES) * 16);
    L.prb_blk = take((nblocks + 1) * 4);
    L.prb_cell = take(size_t(LBEM_MAX_PROBES) * 4);
    L.prb_slot = take(size_t(LBEM_MAX_PROBES) * 4);
    L.flx_cell = take(size_t(LBEM_MAX_FLUX_CELLS) * 4);
    L.flags = take(64);
    L.total = off;
    return L;
}
}  // namespace lbem

// The exported functions below get C linkage from their declarations in lbem.h.

int32_t lbem_version(void) { return 10000; }

const char *lbem_last_error(void) { return g_err; }

lbem_status lbem_workspace_size(const lbem_desc *desc, size_t *bytes) {
    lbem_status st = check_desc(desc);
    if (st) return st;
    if (!bytes) return fail(LBEM_EINVAL, "bytes is NULL");
    *bytes = layout(desc).total;
    return LBEM_OK;
}

size_t lbem_workspace_bytes(const lbem_desc *desc) {
    size_t bytes = 0;
    return lbem_workspace_size(desc, &bytes) == LBEM_OK ? bytes : 0;
}

lbem_status lbem_state_size(const lbem_desc *desc, size_t *bytes) {
    lbem_status st = check_desc(desc);
    if (st) return st;
    if (!bytes) return fail(LBEM_EINVAL, "bytes is NULL");
    *bytes = state_bytes(desc);
    return LBEM_OK;
}

static uint32_t grid_for(size_t n) { return uint32_t((n + kBlock - 1) / kBlock); }

lbem_status lbem_create(const lbem_desc *desc, const float *eps_r, const float *mu_r, const float *sigma,
                        void *workspace, size_t workspace_bytes, void *stream, lbem_lattice **out) {
    lbem_status st = check_desc(desc);
    if (st) return st;
    if (!out) return fail(LBEM_EINVAL, "out is NULL");
    if (!workspace) return fail(LBEM_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(LBEM_EINVAL, "workspace must be 256-byte aligned");
    WsLayout L = layout(desc);
    if (workspace_bytes < L.total)
        return fail(LBEM_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    auto *lat = new (std::nothrow) lbem_lattice();
    if (!lat) return fail(LBEM_ENOMEM, "host allocation failed");
    lat->d = *desc;
    lat->Q = model_pops(desc->model);
    lat->sbytes = storage_bytes(desc->storage);
    lat->N = uint32_t(size_t(desc->nx) * desc->ny * desc->nz);
    lat->bu = row_block(desc) ? uint32_t(desc->nx) : uint32_t(kBlock);
    lat->nblocks = uint32_t((size_t(lat->N) + lat->bu - 1) / lat->bu);
    lat->nobs = grid_for(lat->N);
    lat->scale = (is_f16(desc->storage) && desc->storage_scale != 0.0) ? float(desc->storage_scale) : 1.0f;
    lat->inv_scale = 1.0f / lat->scale;
    lat->stream = static_cast<hipStream_t>(stream);
    lat->ws = static_cast<char *>(workspace);
    lat->ws_bytes = workspace_bytes;
    if (hipGetDevice(&lat->device) != hipSuccess) {
        delete lat;
        return fail(LBEM_EHIP, "hipGetDevice failed");
    }
    lat->L = L;
    lat->pl = pop_layout(desc);
    lat->plane_z = -1;
    lat->det_z = -1;
    lat->t = 0;
    // default launch tuning (measured on MI355X at 256^3): early store
    // addresses for FP32 storage, late ones for the 16-bit formats, hardware
    // block order, no occupancy cap
    lat->tune_form[0] = lat->tune_form[1] = desc->storage == LBEM_F32 ? 0 : 1;
    lat->tune_cap[0] = lat->tune_cap[1] = 0;
    lat->tune_pad[0] = lat->tune_pad[1] = 0;
    hipStream_t s = lat->stream;
    float *eps = reinterpret_cast<float *>(lat->ws + L.eps);
    float *mu = reinterpret_cast<float *>(lat->ws + L.mu);
    float *sig = reinterpret_cast<float *>(lat->ws + L.sig);
    const uint32_t g = grid_for(lat->N);
    hipLaunchKernelGGL(fill_or_copy, dim3(g), dim3(kBlock), 0, s, eps, eps_r, 1.0f, lat->N);
    hipLaunchKernelGGL(fill_or_copy, dim3(g), dim3(kBlock), 0, s, mu, mu_r, 1.0f, lat->N);
    hipLaunchKernelGGL(fill_or_copy, dim3(g), dim3(kBlock), 0, s, sig, sigma, 0.0f, lat->N);
    // zero everything after the media (partials, tables, flags) and the populations
    const size_t tail = L.total - L.en_part;
    hipLaunchKernelGGL(zero_bytes, dim3(grid_for(tail / 4)), dim3(kBlock), 0, s,
                       reinterpret_cast<uint32_t *>(lat->ws + L.en_part), tail / 4);
    // populations and record planes (zero records: phi = 0, so the state is zero)
    const size_t popw = (L.eps - L.pop) / 4;
    hipLaunchKernelGGL(zero_bytes, dim3(grid_for(popw)), dim3(kBlock), 0, s,
                       reinterpret_cast<uint32_t *>(lat->ws + L.pop), popw);
    int32_t *flags = reinterpret_cast<int32_t *>(lat->ws + L.flags);
    hipLaunchKernelGGL(validate_media, dim3(g), dim3(kBlock), 0, s, eps, mu, sig, lat->N, desc->model, flags);
    int32_t counts[4] = {0, 0, 0, 0};
    st = hip_check(hipGetLastError(), "launch");
    if (!st) st = hip_check(hipMemcpyAsync(counts, flags, sizeof(counts), hipMemcpyDeviceToHost, s), "copy flags");
    if (!st) st = hip_check(hipStreamSynchronize(s), "synchronise");
    if (!st && counts[0]) st = fail(LBEM_ENOTFINITE, "%d cells have non-finite media", counts[0]);
    if (!st && counts[1]) st = fail(LBEM_EINVAL, "%d cells have eps_r <= 0, mu_r <= 0 or sigma < 0", counts[1]);
    if (!st && counts[2])
        st = fail(LBEM_EUNSTABLE, "%d cells have eps_r * mu_r < 1 (faster than the vacuum speed)", counts[2]);
    if (!st && counts[3]) st = fail(LBEM_EUNSTABLE, "%d cells have sigma / (3 eps_r) >= 2 (HV current)", counts[3]);
    if (st) {
        delete lat;
        return st;
    }
    *out = lat;
    return LBEM_OK;
}

lbem_status lbem_destroy(lbem_lattice *lat) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    delete lat;
    return LBEM_OK;
}

lbem_status lbem_set_stream(lbem_lattice *lat, void *stream) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    lat->stream = static_cast<hipStream_t>(stream);
    return LBEM_OK;
}

// record plane read by the step at time level t (shifted storage)
static char *read_rec(const lbem_lattice *lat, int64_t t) {
    return lat->ws + lat->L.rec + size_t((t + 1) & 1) * lat->N * kRecBytes;
}

template <class M, class ST>
static void launch_init(lbem_lattice *lat, const float *E, const float *B) {
    const float *eps = reinterpret_cast<const float *>(lat->ws + lat->L.eps);
    const float *mu = reinterpret_cast<const float *>(lat->ws + lat->L.mu);
    char *rec = ST::kShift ? read_rec(lat, 0) : nullptr;
    if (ST::kShift)
        hipLaunchKernelGGL(init_record_kernel, dim3(lat->nobs), dim3(kBlock), 0, lat->stream, rec, eps, mu, E, B, lat->N);
    hipLaunchKernelGGL((init_kernel<M, ST>), dim3(lat->nobs), dim3(kBlock), 0, lat->stream, lat->ws + lat->L.pop,
                       lat->pl, eps, mu, E, B, uint32_t(lat->d.nx), uint32_t(lat->d.ny), uint32_t(lat->d.nz), lat->N,
                       lat->scale, rec);
}

template <class M>
static void dispatch_init(lbem_lattice *lat, const float *E, const float *B) {
    switch (lat->d.storage) {
        case LBEM_F32: launch_init<M, StF32>(lat, E, B); break;
        case LBEM_BF16: launch_init<M, StBF16>(lat, E, B); break;
        case LBEM_F16: launch_init<M, StF16>(lat, E, B); break;
        case LBEM_BF16_SHIFTED: launch_init<M, StBF16S>(lat, E, B); break;
        default: launch_init<M, StF16S>(lat, E, B); break;
    }
}

lbem_status lbem_set_fields(lbem_lattice *lat, const float *E, const float *B) {
    if (!lat || !E || !B) return fail(LBEM_EINVAL, "null argument");
    if (lat->d.model == LBEM_MM) dispatch_init<MM>(lat, E, B);
    else if (lat->d.model == LBEM_MM_DIFF) dispatch_init<MMD>(lat, E, B);
    else dispatch_init<HV>(lat, E, B);
    lat->t = 0;
    return hip_check(hipGetLastError(), "init launch");
}

// Build per-block [start, end) ranges into a cell-sorted list.
static std::vector<int32_t> block_ranges(const std::vector<int32_t> &sorted_cells, uint32_t nblocks, uint32_t bu) {
    std::vector<int32_t> r(nblocks + 1);
    size_t k = 0;
    for (uint32_t b = 0; b <= nblocks; ++b) {
        const int64_t first = int64_t(b) * bu;
        while (k < sorted_cells.size() && sorted_cells[k] < first) ++k;
        r[b] = int32_t(k);
    }
    return r;
}

// Upload the lattice's source list (sorted by cell, per-block ranges).
static lbem_status upload_sources(lbem_lattice *lat) {
    const int32_t n = int32_t(lat->src_cells.size());
    if (n == 0) {
        lat->nsrc = 0;
        return LBEM_OK;
    }
    std::vector<int32_t> order(n);
    for (int32_t k = 0; k < n; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return lat->src_cells[a] < lat->src_cells[b]; });
    std::vector<int32_t> sc(n);
    std::vector<float> sj(3 * size_t(n));
    std::vector<double> tp(2 * size_t(n));
    for (int32_t k = 0; k < n; ++k) {
        const int32_t o = order[k];
        sc[k] = lat->src_cells[o];
        for (int a = 0; a < 3; ++a) sj[3 * k + a] = lat->src_J0[3 * size_t(o) + a];
        tp[2 * k] = lat->src_tp[2 * size_t(o)];
        tp[2 * k + 1] = lat->src_tp[2 * size_t(o) + 1];
    }
    std::vector<int32_t> br = block_ranges(sc, lat->nblocks, lat->bu);
    hipStream_t s = lat->stream;
    lbem_status st = hip_check(hipMemcpyAsync(lat->ws + lat->L.src_blk, br.data(), br.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipMemcpyAsync(lat->ws + lat->L.src_cell, sc.data(), sc.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipMemcpyAsync(lat->ws + lat->L.src_J0, sj.data(), sj.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipMemcpyAsync(lat->ws + lat->L.src_tp, tp.data(), tp.size() * 8, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipStreamSynchronize(s), "synchronise");
    if (!st) lat->nsrc = n;
    return st;
}

static lbem_status check_source(const lbem_lattice *lat, int64_t cell, const float *J0, double period, double phase) {
    if (cell < 0 || cell >= int64_t(lat->N)) return fail(LBEM_EINVAL, "source cell %lld out of range", (long long)cell);
    if (!std::isfinite(J0[0]) || !std::isfinite(J0[1]) || !std::isfinite(J0[2]))
        return fail(LBEM_ENOTFINITE, "source amplitude is not finite");
    if (!(period > 0.0) || !std::isfinite(period) || !std::isfinite(phase))
        return fail(LBEM_EINVAL, "period must be finite and > 0, phase finite");
    return LBEM_OK;
}

lbem_status lbem_set_current_source(lbem_lattice *lat, int32_t n, const int64_t *cells, const float *J0,
                                    double period, double phase) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (n < 0 || n > LBEM_MAX_SOURCES) return fail(LBEM_EINVAL, "source count %d outside [0, %d]", n, LBEM_MAX_SOURCES);
    if (n > 0 && (!cells || !J0)) return fail(LBEM_EINVAL, "null source arrays");
    std::vector<int32_t> sc(n);
    for (int32_t k = 0; k < n; ++k) {
        lbem_status st = check_source(lat, cells[k], J0 + 3 * size_t(k), period, phase);
        if (st) return st;
        sc[k] = int32_t(cells[k]);
    }
    std::vector<int32_t> sorted = sc;
    std::sort(sorted.begin(), sorted.end());
    for (int32_t k = 1; k < n; ++k)
        if (sorted[k] == sorted[k - 1]) return fail(LBEM_EINVAL, "source cell %d repeated", sorted[k]);
    lat->src_cells = sc;
    lat->src_J0.assign(J0, J0 + 3 * size_t(n));
    lat->src_tp.resize(2 * size_t(n));
    for (int32_t k = 0; k < n; ++k) {
        lat->src_tp[2 * size_t(k)] = period;
        lat->src_tp[2 * size_t(k) + 1] = phase;
    }
    return upload_sources(lat);
}

lbem_status lbem_add_point_current(lbem_lattice *lat, int32_t x, int32_t y, int32_t z, const float *J0, double period,
                                   double phase) {
    if (!lat || !J0) return fail(LBEM_EINVAL, "null argument");
    if (x < 0 || y < 0 || z < 0 || x >= lat->d.nx || y >= lat->d.ny || z >= lat->d.nz)
        return fail(LBEM_EINVAL, "cell (%d, %d, %d) outside the lattice", x, y, z);
    if (lat->src_cells.size() >= size_t(LBEM_MAX_SOURCES)) return fail(LBEM_EINVAL, "too many sources");
    const int64_t cell = int64_t(x) + int64_t(lat->d.nx) * (int64_t(y) + int64_t(lat->d.ny) * z);
    lbem_status st = check_source(lat, cell, J0, period, phase);
    if (st) return st;
    for (int32_t c : lat->src_cells)
        if (c == int32_t(cell)) return fail(LBEM_EINVAL, "cell (%d, %d, %d) already has a source", x, y, z);
    lat->src_cells.push_back(int32_t(cell));
    for (int a = 0; a < 3; ++a) lat->src_J0.push_back(J0[a]);
    lat->src_tp.push_back(period);
    lat->src_tp.push_back(phase);
    st = upload_sources(lat);
    if (st) {  // keep the host list equal to what the device holds
        lat->src_cells.pop_back();
        lat->src_J0.resize(lat->src_J0.size() - 3);
        lat->src_tp.resize(lat->src_tp.size() - 2);
    }
    return st;
}

lbem_status lbem_set_plane_source(lbem_lattice *lat, int32_t z, const float *E0, const float *B0, double period) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (z < 0) {
        lat->plane_z = -1;
        return LBEM_OK;
    }
    if (z >= lat->d.nz) return fail(LBEM_EINVAL, "plane z = %d outside the lattice", z);
    if (!E0 || !B0) return fail(LBEM_EINVAL, "null source vectors");
    if (!(period > 0.0) || !std::isfinite(period)) return fail(LBEM_EINVAL, "period must be finite and > 0");
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(E0[a]) || !std::isfinite(B0[a])) return fail(LBEM_ENOTFINITE, "source vector not finite");
        lat->pE0[a] = E0[a];
        lat->pB0[a] = B0[a];
    }
    lat->plane_z = z;
    lat->plane_period = period;
    return LBEM_OK;
}

lbem_status lbem_set_probes(lbem_lattice *lat, int32_t n, const int64_t *cells, int64_t cap_rows, double *series) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (n < 0 || n > LBEM_MAX_PROBES) return fail(LBEM_EINVAL, "probe count %d outside [0, %d]", n, LBEM_MAX_PROBES);
    if (n == 0) {
        lat->nprobe = 0;
        return LBEM_OK;
    }
    if (!cells || !series || cap_rows < 1) return fail(LBEM_EINVAL, "null probe arrays or cap_rows < 1");
    std::vector<int32_t> order(n);
    for (int32_t k = 0; k < n; ++k) {
        if (cells[k] < 0 || cells[k] >= int64_t(lat->N)) return fail(LBEM_EINVAL, "probe cell %lld out of range", (long long)cells[k]);
        order[k] = k;
    }
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cells[a] < cells[b]; });
    std::vector<int32_t> pc(n), ps(n);
    for (int32_t k = 0; k < n; ++k) {
        pc[k] = int32_t(cells[order[k]]);
        ps[k] = order[k];
    }
    std::vector<int32_t> br = block_ranges(pc, lat->nblocks, lat->bu);
    hipStream_t s = lat->stream;
    lbem_status st = hip_check(hipMemcpyAsync(lat->ws + lat->L.prb_blk, br.data(), br.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipMemcpyAsync(lat->ws + lat->L.prb_cell, pc.data(), pc.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipMemcpyAsync(lat->ws + lat->L.prb_slot, ps.data(), ps.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipStreamSynchronize(s), "synchronise");
    if (st) return st;
    lat->nprobe = n;
    lat->prb_cap = cap_rows;
    lat->prb_t0 = lat->t;
    lat->prb_series = series;
    return LBEM_OK;
}

lbem_status lbem_set_flux_monitor(lbem_lattice *lat, int32_t n, const int64_t *cells, int64_t n_begin, int64_t n_end,
                                  double *maxflux) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (n < 0 || n > LBEM_MAX_FLUX_CELLS)
        return fail(LBEM_EINVAL, "flux-monitor cell count %d outside [0, %d]", n, LBEM_MAX_FLUX_CELLS);
    if (n == 0) {
        lat->flx_n = 0;
        return LBEM_OK;
    }
    if (!cells || !maxflux) return fail(LBEM_EINVAL, "null flux-monitor arrays");
    std::vector<int32_t> fc(n);
    for (int32_t k = 0; k < n; ++k) {
        if (cells[k] < 0 || cells[k] >= int64_t(lat->N))
            return fail(LBEM_EINVAL, "flux-monitor cell %lld out of range", (long long)cells[k]);
        fc[k] = int32_t(cells[k]);
    }
    hipStream_t s = lat->stream;
    lbem_status st = hip_check(hipMemcpyAsync(lat->ws + lat->L.flx_cell, fc.data(), fc.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipStreamSynchronize(s), "synchronise");
    if (st) return st;
    lat->flx_n = n;
    lat->flx_t0 = n_begin;
    lat->flx_t1 = n_end;
    lat->flx_max = maxflux;
    return LBEM_OK;
}

lbem_status lbem_set_detector(lbem_lattice *lat, int32_t z) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (z >= lat->d.nz) return fail(LBEM_EINVAL, "detector z = %d outside the lattice", z);
    lat->det_acc = nullptr;
    if (z < 0) {
        lat->det_z = -1;
        return LBEM_OK;
    }
    const uint64_t nxy = uint64_t(lat->d.nx) * lat->d.ny;
    lat->det_z = z;
    lat->det_b0 = uint32_t((uint64_t(z) * nxy) / lat->bu);
    lat->det_b1 = uint32_t((uint64_t(z + 1) * nxy - 1) / lat->bu);
    const size_t words = size_t(lat->L.det_cap) * kSegMax * 2;
    hipLaunchKernelGGL(zero_bytes, dim3(grid_for(words)), dim3(kBlock), 0, lat->stream,
                       reinterpret_cast<uint32_t *>(lat->ws + lat->L.det_part), words);
    return hip_check(hipGetLastError(), "zero detector");
}

lbem_status lbem_detector_read(lbem_lattice *lat, double *out) {
    if (!lat || !out) return fail(LBEM_EINVAL, "null argument");
    if (lat->det_z < 0) return fail(LBEM_ESTATE, "no detector plane set");
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(kBlock), 0, lat->stream,
                       reinterpret_cast<const double *>(lat->ws + lat->L.det_part),
                       (lat->det_b1 - lat->det_b0 + 1) * kSegMax, out);
    return hip_check(hipGetLastError(), "detector sum");
}

lbem_status lbem_set_detector_plane(lbem_lattice *lat, int32_t z, double *acc) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (z >= 0 && !acc) return fail(LBEM_EINVAL, "acc is NULL");
    lbem_status st = lbem_set_detector(lat, z);
    if (st || z < 0) return st;
    lat->det_acc = acc;
    hipLaunchKernelGGL(zero_bytes, dim3(1), dim3(kBlock), 0, lat->stream, reinterpret_cast<uint32_t *>(acc),
                       size_t(2));
    return hip_check(hipGetLastError(), "zero detector accumulator");
}

lbem_status lbem_set_energy_series(lbem_lattice *lat, int32_t every, int64_t cap, double *series) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (every <= 0) {
        lat->en_every = 0;
        return LBEM_OK;
    }
    if (!series || cap < 1) return fail(LBEM_EINVAL, "null energy series or cap < 1");
    lat->en_every = every;
    lat->en_cap = cap;
    lat->en_t0 = lat->t;
    lat->en_series = series;
    return LBEM_OK;
}

// Kernel of a lattice with x extent RB for a tuning choice: form 0 / 1 = the
// row form with LDS x-shifts and early / late store addresses, 2 = the row
// form with direct x-shifted addressing (late addresses), 3 = the same with
// each row split into workgroups of kSegThreads threads.
template <class M, int ODD, class ST, int RB>
static const void *row_kernel_ptr(int form) {
    switch (form) {
        case 0: return reinterpret_cast<const void *>(&row_step_kernel<M, ODD, ST, RB, 0, 0>);
        case 1: return reinterpret_cast<const void *>(&row_step_kernel<M, ODD, ST, RB, 1, 0>);
        case 2: return reinterpret_cast<const void *>(&row_step_kernel<M, ODD, ST, RB, 1, 1>);
        default:
            if constexpr (RB > kSegThreads)
                return reinterpret_cast<const void *>(&row_step_kernel<M, ODD, ST, RB, 1, 1, kSegThreads>);
            else return reinterpret_cast<const void *>(&row_step_kernel<M, ODD, ST, RB, 1, 1>);
    }
}

template <class M, int ODD, class ST>
static const void *step_kernel_ptr(uint32_t rb, int form) {
    switch (rb) {
        case 128: return row_kernel_ptr<M, ODD, ST, 128>(form);
        case 256: return row_kernel_ptr<M, ODD, ST, 256>(form);
        case 384: return row_kernel_ptr<M, ODD, ST, 384>(form);
        case 512: return row_kernel_ptr<M, ODD, ST, 512>(form);
        default: return reinterpret_cast<const void *>(&step_kernel<M, ODD, ST>);
    }
}

template <class M, int ODD>
static const void *step_kernel_ptr_st(const lbem_lattice *lat, int form) {
    const uint32_t rb = row_block(&lat->d);
    switch (lat->d.storage) {
        case LBEM_F32: return step_kernel_ptr<M, ODD, StF32>(rb, form);
        case LBEM_BF16: return step_kernel_ptr<M, ODD, StBF16>(rb, form);
        case LBEM_F16: return step_kernel_ptr<M, ODD, StF16>(rb, form);
        case LBEM_BF16_SHIFTED: return step_kernel_ptr<M, ODD, StBF16S>(rb, form);
        default: return step_kernel_ptr<M, ODD, StF16S>(rb, form);
    }
}

static const void *step_kernel_of(const lbem_lattice *lat, int odd, int form) {
    if (lat->d.model == LBEM_MM) return odd ? step_kernel_ptr_st<MM, 1>(lat, form) : step_kernel_ptr_st<MM, 0>(lat, form);
    if (lat->d.model == LBEM_MM_DIFF)
        return odd ? step_kernel_ptr_st<MMD, 1>(lat, form) : step_kernel_ptr_st<MMD, 0>(lat, form);
    return odd ? step_kernel_ptr_st<HV, 1>(lat, form) : step_kernel_ptr_st<HV, 0>(lat, form);
}

// Dynamic LDS that caps the resident blocks per compute unit at `cap`
// (0: no cap), given the kernel's static LDS.
size_t lbem::lds_pad_for(const void *kernel, int cap) {
    if (cap <= 0) return 0;
    hipFuncAttributes attr{};
    if (hipFuncGetAttributes(&attr, kernel) != hipSuccess) return 0;
    int dev = 0, lds_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds_cu <= 0)
        return 0;
    int lds_block = 0;  // per-workgroup limit (160 KB on gfx950)
    if (hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        size_t(lds_block) <= attr.sharedSizeBytes)
        return 0;
    const size_t per_block = size_t(lds_cu) / size_t(cap + 1) + 1;  // cap blocks fit, cap + 1 do not
    const size_t need = per_block > attr.sharedSizeBytes ? per_block - attr.sharedSizeBytes : 0;
    return std::min<size_t>(need, size_t(lds_block) - attr.sharedSizeBytes);
}

uint32_t lbem::step_segments(const lbem_lattice *lat, int odd) {
    const uint32_t rb = row_block(&lat->d);
    return ((lat->tune_form[odd] & 3) == 3 && rb > uint32_t(kSegThreads)) ? rb / kSegThreads : 1u;
}

void lbem::dispatch_step(const lbem_lattice *lat, const StepArgs &a, int odd) {
    const void *k = step_kernel_of(lat, odd, lat->tune_form[odd] & 3);
    const uint32_t rb = row_block(&lat->d), seg = step_segments(lat, odd);
    StepArgs b = a;
    // grouped order: one layout chunk of rows (at least 16 rows) per group
    const uint32_t rows_per_group = lat->pl.rshift < 31 ? std::max(16u, 1u << lat->pl.rshift) : 16u;
    b.xcd_group = (lat->tune_form[odd] >> 2) & 1 ? rows_per_group * seg : 0u;
    void *args[] = {&b};
    (void)hipLaunchKernel(k, dim3(lat->nblocks * seg), dim3(rb ? rb / seg : kBlock), args, lat->tune_pad[odd],
                          lat->stream);
}


StepArgs lbem::base_step_args(lbem_lattice *lat) {
    const WsLayout &L = lat->L;
    StepArgs a{};
    a.pop = lat->ws + L.pop;
    a.pl = lat->pl;
    a.eps = reinterpret_cast<const float *>(lat->ws + L.eps);
    a.mu = reinterpret_cast<const float *>(lat->ws + L.mu);
    a.sig = reinterpret_cast<const float *>(lat->ws + L.sig);
    a.nx = lat->d.nx;
    a.ny = lat->d.ny;
    a.nz = lat->d.nz;
    a.N = lat->N;
    a.scale = lat->scale;
    a.inv_scale = lat->inv_scale;
    if (lat->nsrc > 0) {
        a.src_blk = reinterpret_cast<const int32_t *>(lat->ws + L.src_blk);
        a.src_cell = reinterpret_cast<const int32_t *>(lat->ws + L.src_cell);
        a.src_J0 = reinterpret_cast<const float *>(lat->ws + L.src_J0);
        a.src_tp = reinterpret_cast<const double *>(lat->ws + L.src_tp);
    }
    a.plane_z = lat->plane_z;
    a.det_z = -1;
    if (shifted(lat->d.storage)) {
        a.rec[0] = lat->ws + L.rec;
        a.rec[1] = lat->ws + L.rec + size_t(lat->N) * kRecBytes;
    }
    return a;
}

lbem_status lbem_step(lbem_lattice *lat, int64_t nsteps) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (nsteps < 0) return fail(LBEM_EINVAL, "nsteps < 0");
    return step_impl(lat, nsteps, nullptr);
}

static void launch_flux(const lbem_lattice *lat);

lbem_status lbem::step_impl(lbem_lattice *lat, int64_t nsteps, float *frames) {
    const WsLayout &L = lat->L;
    StepArgs a = base_step_args(lat);
    if (lat->nprobe > 0) {
        a.prb_blk = reinterpret_cast<const int32_t *>(lat->ws + L.prb_blk);
        a.prb_cell = reinterpret_cast<const int32_t *>(lat->ws + L.prb_cell);
        a.prb_slot = reinterpret_cast<const int32_t *>(lat->ws + L.prb_slot);
    }
    a.det_z = lat->det_z;
    if (lat->det_z >= 0) {
        a.det_b0 = lat->det_b0;
        a.det_b1 = lat->det_b1;
        a.det_part = reinterpret_cast<double *>(lat->ws + L.det_part);
    }
    double *en_part = reinterpret_cast<double *>(lat->ws + L.en_part);
    for (int64_t s = 0; s < nsteps; ++s) {
        const int64_t t = lat->t;
        a.src_t = double(t);
        if (lat->plane_z >= 0) {
            const double w = source_weight(double(t), lat->plane_period, 0.0);
            for (int k = 0; k < 3; ++k) {
                a.Eimp[k] = float(lat->pE0[k] * w);
                a.Bimp[k] = float(lat->pB0[k] * w);
            }
        }
        if (lat->nprobe > 0) a.prb_row = lat->prb_series + ((t - lat->prb_t0) % lat->prb_cap) * lat->nprobe * 6;
        const bool en = lat->en_every > 0 && (t - lat->en_t0) % lat->en_every == 0;
        a.en_part = en ? en_part : nullptr;
        a.E_out = frames ? frames + size_t(s) * 3 * lat->N : nullptr;
        if (lat->flx_n > 0 && t >= lat->flx_t0 && t < lat->flx_t1) launch_flux(lat);
        dispatch_step(lat, a, int(t & 1));
        if (en) {
            double *dst = lat->en_series + ((t - lat->en_t0) / lat->en_every) % lat->en_cap;
            hipLaunchKernelGGL(sum_partials, dim3(1), dim3(kBlock), 0, lat->stream, en_part,
                               lat->nblocks * step_segments(lat, int(t & 1)), dst);
        }
        lbem_status st = hip_check(hipGetLastError(), "step launch");
        if (st) return st;
        lat->t = t + 1;
    }
    if (lat->det_acc && lat->det_z >= 0 && nsteps > 0) return lbem_detector_read(lat, lat->det_acc);
    return LBEM_OK;
}

lbem_status lbem_get_time(lbem_lattice *lat, int64_t *t) {
    if (!lat || !t) return fail(LBEM_EINVAL, "null argument");
    *t = lat->t;
    return LBEM_OK;
}

template <class M, int ODD, class ST>
static void launch_obs(const ObsArgs &a, uint32_t nblocks, hipStream_t s) {
    hipLaunchKernelGGL((observe_kernel<M, ODD, ST>), dim3(nblocks), dim3(kBlock), 0, s, a);
}
template <class M, int ODD>
static void dispatch_obs_storage(const lbem_lattice *lat, const ObsArgs &a) {
    switch (lat->d.storage) {
        case LBEM_F32: launch_obs<M, ODD, StF32>(a, lat->nobs, lat->stream); break;
        case LBEM_BF16: launch_obs<M, ODD, StBF16>(a, lat->nobs, lat->stream); break;
        case LBEM_F16: launch_obs<M, ODD, StF16>(a, lat->nobs, lat->stream); break;
        case LBEM_BF16_SHIFTED: launch_obs<M, ODD, StBF16S>(a, lat->nobs, lat->stream); break;
        default: launch_obs<M, ODD, StF16S>(a, lat->nobs, lat->stream); break;
    }
}

static ObsArgs obs_args(const lbem_lattice *lat) {
    const WsLayout &L = lat->L;
    ObsArgs a{};
    a.pop = lat->ws + L.pop;
    a.pl = lat->pl;
    a.eps = reinterpret_cast<const float *>(lat->ws + L.eps);
    a.mu = reinterpret_cast<const float *>(lat->ws + L.mu);
    a.sig = reinterpret_cast<const float *>(lat->ws + L.sig);
    a.nx = lat->d.nx;
    a.ny = lat->d.ny;
    a.nz = lat->d.nz;
    a.N = lat->N;
    a.bu = lat->bu;
    a.inv_scale = lat->inv_scale;
    if (lat->nsrc > 0) {
        a.src_blk = reinterpret_cast<const int32_t *>(lat->ws + L.src_blk);
        a.src_cell = reinterpret_cast<const int32_t *>(lat->ws + L.src_cell);
        a.src_J0 = reinterpret_cast<const float *>(lat->ws + L.src_J0);
        a.src_tp = reinterpret_cast<const double *>(lat->ws + L.src_tp);
        a.src_t = double(lat->t);
    }
    if (shifted(lat->d.storage)) a.rec = read_rec(lat, lat->t);
    return a;
}

template <class M, int ODD>
static void launch_flux_st(const lbem_lattice *lat, const ObsArgs &a) {
    const int32_t *cells = reinterpret_cast<const int32_t *>(lat->ws + lat->L.flx_cell);
    const uint32_t n = uint32_t(lat->flx_n);
    const dim3 g((n + kBlock - 1) / kBlock), b(kBlock);
    switch (lat->d.storage) {
        case LBEM_F32: hipLaunchKernelGGL((flux_kernel<M, ODD, StF32>), g, b, 0, lat->stream, a, cells, n, lat->flx_max); break;
        case LBEM_BF16: hipLaunchKernelGGL((flux_kernel<M, ODD, StBF16>), g, b, 0, lat->stream, a, cells, n, lat->flx_max); break;
        case LBEM_F16: hipLaunchKernelGGL((flux_kernel<M, ODD, StF16>), g, b, 0, lat->stream, a, cells, n, lat->flx_max); break;
        case LBEM_BF16_SHIFTED:
            hipLaunchKernelGGL((flux_kernel<M, ODD, StBF16S>), g, b, 0, lat->stream, a, cells, n, lat->flx_max);
            break;
        default: hipLaunchKernelGGL((flux_kernel<M, ODD, StF16S>), g, b, 0, lat->stream, a, cells, n, lat->flx_max); break;
    }
}

// Fold |E x H| of the current state into the monitor's maxima.
static void launch_flux(const lbem_lattice *lat) {
    const ObsArgs a = obs_args(lat);
    const int odd = int(lat->t & 1);
    if (lat->d.model == LBEM_MM) {
        if (odd) launch_flux_st<MM, 1>(lat, a);
        else launch_flux_st<MM, 0>(lat, a);
    } else if (lat->d.model == LBEM_MM_DIFF) {
        if (odd) launch_flux_st<MMD, 1>(lat, a);
        else launch_flux_st<MMD, 0>(lat, a);
    } else {
        if (odd) launch_flux_st<HV, 1>(lat, a);
        else launch_flux_st<HV, 0>(lat, a);
    }
}

static lbem_status observe(lbem_lattice *lat, float *E, float *B, float *D, float *H, double *en_part) {
    ObsArgs a = obs_args(lat);
    a.E = E;
    a.B = B;
    a.D = D;
    a.H = H;
    a.en_part = en_part;
    const int odd = int(lat->t & 1);
    if (lat->d.model == LBEM_MM) {
        if (odd) dispatch_obs_storage<MM, 1>(lat, a);
        else dispatch_obs_storage<MM, 0>(lat, a);
    } else if (lat->d.model == LBEM_MM_DIFF) {
        if (odd) dispatch_obs_storage<MMD, 1>(lat, a);
        else dispatch_obs_storage<MMD, 0>(lat, a);
    } else {
        if (odd) dispatch_obs_storage<HV, 1>(lat, a);
        else dispatch_obs_storage<HV, 0>(lat, a);
    }
    return hip_check(hipGetLastError(), "observe launch");
}

lbem_status lbem_get_fields(lbem_lattice *lat, float *E, float *B, float *D, float *H) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    return observe(lat, E, B, D, H, nullptr);
}

lbem_status lbem_energy(lbem_lattice *lat, double *out) {
    if (!lat || !out) return fail(LBEM_EINVAL, "null argument");
    double *part = reinterpret_cast<double *>(lat->ws + lat->L.en_part);
    lbem_status st = observe(lat, nullptr, nullptr, nullptr, nullptr, part);
    if (st) return st;
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(kBlock), 0, lat->stream, part, lat->nobs, out);
    return hip_check(hipGetLastError(), "energy sum");
}

lbem_status lbem_check(lbem_lattice *lat, double max_energy, double *energy) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (!(max_energy >= 0.0)) return fail(LBEM_EINVAL, "max_energy must be >= 0 (0: no bound)");
    // the two FP64 results go to the flags block of the workspace (its first
    // 16 bytes hold the media validation counts)
    double *dev = reinterpret_cast<double *>(lat->ws + lat->L.flags + 16);
    lbem_status st = lbem_energy(lat, dev);
    if (!st && lat->det_z >= 0) st = lbem_detector_read(lat, dev + 1);
    double host[2] = {0.0, 0.0};
    if (!st) st = hip_check(hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, lat->stream), "copy check");
    if (!st) st = hip_check(hipStreamSynchronize(lat->stream), "synchronise");
    if (st) return st;
    if (lat->det_z < 0) host[1] = 0.0;
    if (energy) *energy = host[0];
    if (!std::isfinite(host[0]))
        return fail(LBEM_ENOTFINITE, "the field energy at time level %lld is not finite", (long long)lat->t);
    if (!std::isfinite(host[1]))
        return fail(LBEM_ENOTFINITE, "the detector sum at time level %lld is not finite", (long long)lat->t);
    if (max_energy > 0.0 && host[0] > max_energy)
        return fail(LBEM_EUNSTABLE, "the field energy %.6e at time level %lld exceeds the bound %.6e", host[0],
                    (long long)lat->t, max_energy);
    return LBEM_OK;
}

// state = populations, then (shifted storage) the record plane the next step reads
static lbem_status copy_state(lbem_lattice *lat, void *dst, const void *src, int64_t t) {
    const size_t pb = pop_bytes(&lat->d), rb = state_bytes(&lat->d) - pb;
    char *pop = lat->ws + lat->L.pop, *rec = read_rec(lat, t);
    char *d = static_cast<char *>(dst);
    const char *sr = static_cast<const char *>(src);
    lbem_status st = hip_check(hipMemcpyAsync(d ? d : pop, d ? pop : sr, pb, hipMemcpyDeviceToDevice, lat->stream),
                               "copy state");
    if (!st && rb)
        st = hip_check(hipMemcpyAsync(d ? d + pb : rec, d ? rec : sr + pb, rb, hipMemcpyDeviceToDevice, lat->stream),
                       "copy records");
    return st;
}

lbem_status lbem_save_state(lbem_lattice *lat, void *dst) {
    if (!lat || !dst) return fail(LBEM_EINVAL, "null argument");
    return copy_state(lat, dst, nullptr, lat->t);
}

lbem_status lbem_load_state(lbem_lattice *lat, const void *src, int64_t t) {
    if (!lat || !src) return fail(LBEM_EINVAL, "null argument");
    if (t < 0) return fail(LBEM_EINVAL, "time level < 0");
    lbem_status st = copy_state(lat, nullptr, src, t);
    if (st) return st;
    lat->t = t;
    return LBEM_OK;
}

lbem_status lbem_set_tuning(lbem_lattice *lat, const int32_t *form, const int32_t *blocks_per_cu) {
    if (!lat || !form || !blocks_per_cu) return fail(LBEM_EINVAL, "null argument");
    for (int p = 0; p < 2; ++p) {
        if (form[p] < 0 || form[p] > 7)
            return fail(LBEM_EINVAL, "form must be 0, 1, 2 or 3, plus 4 for the grouped XCD order");
        if (blocks_per_cu[p] < 0 || blocks_per_cu[p] > 64) return fail(LBEM_EINVAL, "blocks_per_cu must be in [0, 64]");
    }
    for (int p = 0; p < 2; ++p) {
        lat->tune_form[p] = form[p];
        lat->tune_cap[p] = blocks_per_cu[p];
        lat->tune_pad[p] = lds_pad_for(step_kernel_of(lat, p, form[p] & 3), blocks_per_cu[p]);
    }
    return LBEM_OK;
}

lbem_status lbem_get_tuning(lbem_lattice *lat, int32_t *form, int32_t *blocks_per_cu) {
    if (!lat || !form || !blocks_per_cu) return fail(LBEM_EINVAL, "null argument");
    for (int p = 0; p < 2; ++p) {
        form[p] = lat->tune_form[p];
        blocks_per_cu[p] = lat->tune_cap[p];
    }
    return LBEM_OK;
}

lbem_status lbem_autotune(lbem_lattice *lat, int32_t trial_steps, void *backup) {
    if (!lat || !backup) return fail(LBEM_EINVAL, "null argument");
    if (trial_steps < 1) return fail(LBEM_EINVAL, "trial_steps must be >= 1");
    lbem_status st = copy_state(lat, backup, nullptr, lat->t);
    if (st) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    st = hip_check(hipEventCreate(&e0), "event");
    if (!st) st = hip_check(hipEventCreate(&e1), "event");
    static const int caps[] = {0, 2, 3, 4};
    // every candidate times one parity's kernel alone; the data it leaves is
    // not a valid state, which is why the state is restored afterwards
    const StepArgs a = base_step_args(lat);
    struct Cand {
        int32_t form, cap;
        float ms;
    };
    // milliseconds of `launches` launches of one parity under (form, cap)
    auto time_cand = [&](int p, const Cand &c, int launches, float &ms) {
        int32_t f2[2] = {lat->tune_form[0], lat->tune_form[1]}, c2[2] = {lat->tune_cap[0], lat->tune_cap[1]};
        f2[p] = c.form;
        c2[p] = c.cap;
        lbem_status s2 = lbem_set_tuning(lat, f2, c2);
        if (s2) return s2;
        dispatch_step(lat, a, p);  // warm-up
        s2 = hip_check(hipEventRecord(e0, lat->stream), "record");
        for (int k = 0; k < launches && !s2; ++k) dispatch_step(lat, a, p);
        if (!s2) s2 = hip_check(hipGetLastError(), "trial launch");
        if (!s2) s2 = hip_check(hipEventRecord(e1, lat->stream), "record");
        if (!s2) s2 = hip_check(hipEventSynchronize(e1), "sync");
        if (!s2) s2 = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        return s2;
    };
    for (int p = 0; p < 2 && !st; ++p) {
        // candidate forms: kernels 0-2 (row lattices), 3 (rows longer than a
        // split workgroup), each in both block orders; generic lattices: order only
        const uint32_t rb = row_block(&lat->d);
        std::vector<Cand> cands;
        for (int order = 0; order < 2; ++order)
            for (int k = 0; k < 4; ++k)
                if ((rb && (k < 3 || rb > uint32_t(kSegThreads))) || (!rb && k == 0))
                    for (int cap : caps) cands.push_back({k + 4 * order, cap, 0.f});
        // stage 1: every candidate over trial_steps launches
        for (Cand &c : cands) {
            st = time_cand(p, c, trial_steps, c.ms);
            if (st) break;
        }
        if (st) break;
        // stage 2: the fastest few again, over twice as many launches in
        // alternating rounds, so that one noisy stage-1 timing does not decide
        std::stable_sort(cands.begin(), cands.end(), [](const Cand &x, const Cand &y) { return x.ms < y.ms; });
        const size_t nf = std::min<size_t>(4, cands.size());
        for (size_t i = 0; i < nf; ++i) cands[i].ms = 0.f;
        for (int round = 0; round < 2 && !st; ++round)
            for (size_t i = 0; i < nf && !st; ++i) {
                float ms = 0.f;
                st = time_cand(p, cands[i], 2 * trial_steps, ms);
                cands[i].ms += ms;
            }
        if (st) break;
        size_t best = 0;
        for (size_t i = 1; i < nf; ++i)
            if (cands[i].ms < cands[best].ms) best = i;
        int32_t f2[2] = {lat->tune_form[0], lat->tune_form[1]}, c2[2] = {lat->tune_cap[0], lat->tune_cap[1]};
        f2[p] = cands[best].form;
        c2[p] = cands[best].cap;
        st = lbem_set_tuning(lat, f2, c2);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    lbem_status st2 = copy_state(lat, nullptr, backup, lat->t);
    return st ? st : st2;
}
