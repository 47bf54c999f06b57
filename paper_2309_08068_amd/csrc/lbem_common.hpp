// lbem_common.hpp -- storage formats, neighbour addressing and block reductions
// shared by the step, observation and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbem_model.hpp"

namespace lbem {

constexpr int kBlock = 256;  // threads per block of the lattice kernels (4 waves)
// Per-block detector partials are kept at a stride of kSegMax slots per table
// unit, so that a row may be split into up to kSegMax workgroups.
constexpr int kSegMax = 4;
constexpr int kSegThreads = 128;  // threads per workgroup of a split row

// ------------------------------------------------------------ storage formats
// Populations live in HBM as FP32, BF16 or FP16; collision math is FP32.
// raw<NT>() / put<NT>() move the stored representation (NT: non-temporal
// hint, for streams that are touched once per step); cvt() / pack() convert.
template <class T, bool NT>
__device__ __forceinline__ T raw(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <class T, bool NT>
__device__ __forceinline__ void put(T *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

struct StF32 {
    using T = float;
    static constexpr int kBytes = 4;
    static constexpr bool kShift = false;
    __device__ static float cvt(T r, float) { return r; }
    __device__ static T pack(float v, float) { return v; }
    template <bool NT = false>
    __device__ static float load(const T *p, uint32_t i, float inv) { return cvt(raw<T, NT>(p + i), inv); }
    template <bool NT = false>
    __device__ static void store(T *p, uint32_t i, float v, float scale) { put<T, NT>(p + i, pack(v, scale)); }
};

struct StBF16 {
    using T = uint16_t;
    static constexpr int kBytes = 2;
    static constexpr bool kShift = false;
    __device__ static float cvt(T r, float) { return __uint_as_float(uint32_t(r) << 16); }
    // round to nearest, ties to even (one v_cvt_pk_bf16_f32 on gfx950)
    __device__ static T pack(float v, float) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v)); }
    template <bool NT = false>
    __device__ static float load(const T *p, uint32_t i, float inv) { return cvt(raw<T, NT>(p + i), inv); }
    template <bool NT = false>
    __device__ static void store(T *p, uint32_t i, float v, float scale) { put<T, NT>(p + i, pack(v, scale)); }
};

struct StF16 {
    using T = _Float16;
    static constexpr int kBytes = 2;
    static constexpr bool kShift = false;
    // values are held multiplied by a power-of-two scale
    __device__ static float cvt(T r, float inv_scale) { return float(r) * inv_scale; }
    __device__ static T pack(float v, float scale) { return _Float16(v * scale); }
    template <bool NT = false>
    __device__ static float load(const T *p, uint32_t i, float inv) { return cvt(raw<T, NT>(p + i), inv); }
    template <bool NT = false>
    __device__ static void store(T *p, uint32_t i, float v, float scale) { put<T, NT>(p + i, pack(v, scale)); }
};

// The same 16-bit formats holding equilibrium-shifted populations (see Shift
// in lbem_model.hpp); the kernels add the per-cell record traffic.
struct StBF16S : StBF16 {
    static constexpr bool kShift = true;
};
struct StF16S : StF16 {
    static constexpr bool kShift = true;
};

// ------------------------------------------------------------ launch order
// The hardware hands consecutive workgroups of a grid to the 8 XCDs in turn
// (workgroup b runs on XCD b mod 8), each XCD with its own L2.  The grouped
// order renumbers blocks so that each XCD takes groups of G consecutive blocks
// (group j of the grid goes to XCD j mod 8): neighbouring rows then share an
// L2 (the shifted storage re-reads each record from up to 12 neighbours),
// while the 8 XCDs still sweep nearby addresses.  A bijection of [0, nb); the
// tail that does not fill a round of 8 groups keeps its numbering.
constexpr uint32_t kXCDs = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb, uint32_t G) {
    const uint32_t full = nb / (kXCDs * G) * (kXCDs * G);
    if (b >= full) return b;
    const uint32_t x = b % kXCDs, i = b / kXCDs;  // XCD, and the block's index on it
    return ((i / G) * kXCDs + x) * G + i % G;
}

// ------------------------------------------------------------ population layout
// Cells are grouped into chunks of 2^rshift consecutive x-rows (row = y + ny z);
// a chunk holds all Q population planes of its cells together, so element
// (q, row, x) lives at (row >> rshift) * QC + q * C + (row & mask) * nx + x
// with C cells per chunk and QC = Q * C.  A workgroup's Q streams then lie
// within about a megabyte instead of Q planes spread over the whole state,
// which keeps address translation and DRAM pages local.  A lattice with a
// single chunk (C = N) is the plain [Q][N] layout.
struct PopLayout {
    uint32_t nx, rshift, C;  // x extent, log2 of rows per chunk, cells per chunk (with row padding)
    uint64_t QC;             // elements per chunk
    uint32_t pitch;          // cells from one row of a chunk to the next (>= nx)
    __host__ __device__ uint64_t base(uint32_t row) const {
        return uint64_t(row >> rshift) * QC + uint64_t(row & ((1u << rshift) - 1u)) * pitch;
    }
    __host__ __device__ uint64_t index(int q, uint32_t cell) const {
        const uint32_t row = cell / nx;
        return base(row) + uint64_t(q) * C + (cell - row * nx);
    }
};

// ------------------------------------------------------------ addressing
// Periodic neighbours of one cell: coordinates of x-1, x, x+1 and the row
// offsets of y-1, y, y+1 and z-1, z, z+1.
struct Nbr {
    uint32_t c;
    uint32_t xs[3];
    uint32_t ys[3];
    uint32_t zs[3];
    __device__ __forceinline__ uint32_t at(int dx, int dy, int dz) const {
        return xs[dx + 1] + ys[dy + 1] + zs[dz + 1];
    }
};

__device__ __forceinline__ Nbr make_nbr(uint32_t c, uint32_t x, uint32_t y, uint32_t z, uint32_t nx, uint32_t ny,
                                        uint32_t nz) {
    Nbr n;
    n.c = c;
    const uint32_t nxy = nx * ny;
    n.xs[0] = x == 0 ? nx - 1 : x - 1;
    n.xs[1] = x;
    n.xs[2] = x + 1 == nx ? 0 : x + 1;
    n.ys[0] = (y == 0 ? ny - 1 : y - 1) * nx;
    n.ys[1] = y * nx;
    n.ys[2] = (y + 1 == ny ? 0 : y + 1) * nx;
    n.zs[0] = (z == 0 ? nz - 1 : z - 1) * nxy;
    n.zs[1] = z * nxy;
    n.zs[2] = (z + 1 == nz ? 0 : z + 1) * nxy;
    return n;
}

// In-place AA streaming.  The array holds, before the step at time level t:
//   t even: slot (q, x) = population q at x (natural layout);
//   t odd:  slot (opp q, x - v_q) = population q arriving at x (it is the
//           post-collision value that x - v_q wrote during the previous step).
// The step at an even t writes f'_q(x) to slot (opp q, x); at an odd t it
// writes f'_q(x) to slot (q, x + v_q).  Each cell reads exactly the slots it
// later writes, so the update is race-free without a second array.  The
// aligned even-parity accesses carry the non-temporal hint (each slot is
// touched once per step); the shifted odd-parity accesses of this generic form
// do not, because their cache lines are shared with neighbouring waves.
template <class M, int ODD, class ST>
__device__ __forceinline__ void gather(const typename ST::T *__restrict__ pop, size_t N, const Nbr &nb,
                                       float (&f)[M::Q], float inv_scale) {
#pragma unroll
    for (int q = 0; q < M::Q; ++q) {
        if (ODD) {
            const uint32_t i = nb.at(-M::vel(q, 0), -M::vel(q, 1), -M::vel(q, 2));
            f[q] = ST::load(pop + size_t(M::opp(q)) * N, i, inv_scale);
        } else {
            f[q] = ST::template load<true>(pop + size_t(q) * N, nb.c, inv_scale);
        }
    }
}

// gather for any layout (element indices from PopLayout; used off the hot path)
template <class M, int ODD, class ST>
__device__ __forceinline__ void gather_any(const typename ST::T *__restrict__ pop, const PopLayout &L, const Nbr &nb,
                                           float (&f)[M::Q], float inv_scale) {
#pragma unroll
    for (int q = 0; q < M::Q; ++q) {
        if (ODD) f[q] = ST::cvt(pop[L.index(M::opp(q), nb.at(-M::vel(q, 0), -M::vel(q, 1), -M::vel(q, 2)))], inv_scale);
        else f[q] = ST::cvt(pop[L.index(q, nb.c)], inv_scale);
    }
}

template <class M, int ODD, class ST>
__device__ __forceinline__ void scatter(typename ST::T *__restrict__ pop, size_t N, const Nbr &nb,
                                        const float (&f)[M::Q], float scale) {
#pragma unroll
    for (int q = 0; q < M::Q; ++q) {
        if (ODD) {
            const uint32_t i = nb.at(M::vel(q, 0), M::vel(q, 1), M::vel(q, 2));
            ST::store(pop + size_t(q) * N, i, f[q], scale);
        } else {
            ST::template store<true>(pop + size_t(M::opp(q)) * N, nb.c, f[q], scale);
        }
    }
}

// In-place streaming stores population q where it loaded opp(q), so a
// compiler left alone keeps every load address live until the matching store
// and runs out of registers.  Passing the neighbour table and the base pointer
// through an empty asm statement that also consumes a collision result makes
// them opaque: the store addresses are then formed after the collision.
template <class P>
__device__ __forceinline__ void late_addresses(Nbr &nb, P *&base, float after) {
    asm volatile(""
                 : "+v"(nb.c), "+v"(nb.xs[0]), "+v"(nb.xs[1]), "+v"(nb.xs[2]), "+v"(nb.ys[0]), "+v"(nb.ys[1]),
                   "+v"(nb.ys[2]), "+v"(nb.zs[0]), "+v"(nb.zs[1]), "+v"(nb.zs[2]), "+s"(base)
                 : "v"(after));
}

// ------------------------------------------------------------ shifted storage
// Add back phi_q(R_{x - v_q}) to freshly gathered shifted populations; cell_of
// maps a velocity offset (dx, dy, dz) to the neighbour's cell index.
template <class M, class F>
__device__ __forceinline__ void unshift(float (&f)[M::Q], const u32x4 *__restrict__ rec, F &&cell_of) {
    shift_all<M>(f, 1.f, [&](int k) {
        return rec_unpack(rec[cell_of(-Shift<M>::vel(k, 0), -Shift<M>::vel(k, 1), -Shift<M>::vel(k, 2))]);
    });
}

// Subtract phi_q(R_x) from the post-collision populations of this cell and
// write its record (non-temporal: it is read again only in the next step).
template <class M>
__device__ __forceinline__ void shift_out(float (&f)[M::Q], const float E[3], const float B[3], float eps_r,
                                          float mu_r, u32x4 *__restrict__ rec, uint32_t c, bool store) {
    Rec r;
    const u32x4 w = rec_pack(E, B, eps_r, 1.0f / mu_r, r);
    if (store) __builtin_nontemporal_store(w, rec + c);
    shift_all<M>(f, -1.f, [&](int) { return r; });
}

// ------------------------------------------------------------ row form
// Number of populations of M whose velocity has a non-zero x component.
template <class M>
constexpr int n_xshift() {
    int n = 0;
    for (int q = 0; q < M::Q; ++q) n += M::vel(q, 0) != 0;
    return n;
}

// Workgroup barrier around a phase change of a reused LDS array.  The
// compiler is kept from moving any memory access across it (empty asm with a
// memory clobber on both sides): the backend has been seen to sink LDS reads
// below a plain __syncthreads() under register pressure, after which other
// threads overwrite the array.
__device__ __forceinline__ void lds_phase_barrier() {
    asm volatile("" ::: "memory");
    __syncthreads();
    asm volatile("" ::: "memory");
}

// HBM writes whole 64-byte pieces: a store that covers only part of one
// costs a read-modify-write of the piece.  A row whose byte length is not a
// multiple of this ends in such a piece unless the padding cells after it
// (never read as populations) are written too.
constexpr uint32_t kWritePiece = 64;

// Gather / scatter of the in-place AA streaming for a block that owns one
// whole x-row of nx <= RB cells (y, z uniform; threads past the row idle).
// Every HBM access is the aligned
// row segment of one population plane, with the non-temporal hint; the +-1 x
// shifts of the odd parity go through the LDS array sh[n_xshift][RB], which
// keeps partial cache lines out of the memory traffic.  The direct variant
// (gather_direct / scatter_direct) addresses the shifted cells in HBM instead
// (no LDS; shared cache lines, so no non-temporal hint on those).  Addresses
// are a uniform row base (scalar registers) plus one 32-bit byte offset of x.
template <class M, class ST, int RB>
struct RowIO {
    using T = typename ST::T;
    // global address space kept explicit: a generic pointer that has passed
    // through late() would otherwise turn every access into a flat one
    using gchar = __attribute__((address_space(1))) char;
    gchar *pop;
    PopLayout L;
    uint32_t ny, x, xo, nx;
    bool live;  // x < nx: the row block has RB >= nx threads, those past the row idle
    bool pad;   // an idle thread whose padding cell lies in the row's last kWritePiece bytes
    uint32_t yr[3], zr[3];

    // x: this thread's cell along the row (threadIdx.x unless a row is split
    // over several workgroups); the row length is L.nx <= RB.  An idle thread
    // (x >= nx) computes on a copy of some cell's data and stores nothing of
    // it, except that the idle threads whose own cell is a padding cell in
    // the row's last write piece (below RB <= pitch) store their values there
    // and load from there, so that a row's stores cover whole pieces.  The
    // other idle threads load the row's last cell, which keeps every load
    // outside a branch.  In LDS an idle thread only writes slot RB - 1 >= nx,
    // which no live thread reads (idle threads only exist when nx < RB).
    __device__ RowIO(const void *p, const PopLayout &l, uint32_t ny_, uint32_t nz, uint32_t row,
                     uint32_t x_ = threadIdx.x)
        : pop((gchar *)(p)), L(l), ny(ny_), x(x_ < l.nx ? x_ : l.nx - 1u), nx(l.nx),
          live(x_ < l.nx),
          pad(x_ >= l.nx &&
              x_ * uint32_t(sizeof(T)) < (l.nx * uint32_t(sizeof(T)) + kWritePiece - 1u) / kWritePiece * kWritePiece) {
        xo = (live || pad ? x_ : l.nx - 1u) * uint32_t(sizeof(T));
        const uint32_t y = row % ny_, z = row / ny_;
        yr[0] = y == 0 ? ny_ - 1 : y - 1;
        yr[1] = y;
        yr[2] = y + 1 == ny_ ? 0 : y + 1;
        zr[0] = z == 0 ? nz - 1 : z - 1;
        zr[1] = z;
        zr[2] = z + 1 == nz ? 0 : z + 1;
    }
    __device__ uint32_t row_of(int dy, int dz) const { return yr[dy + 1] + ny * zr[dz + 1]; }
    // x + dx (|dx| <= 1), periodic along the row
    __device__ uint32_t xw(int dx) const {
        return dx > 0 ? (x + 1 >= nx ? 0 : x + 1) : dx < 0 ? (x == 0 ? nx - 1 : x - 1) : x;
    }
    // LDS slot of x + dx for a live thread; idle ones share slot RB - 1
    __device__ uint32_t slot(int dx) const { return live ? xw(dx) : uint32_t(RB - 1); }
    // byte offset of (q, row + (dy, dz), x = 0)
    __device__ uint64_t row_base(int q, int dy, int dz) const {
        return (L.base(row_of(dy, dz)) + uint64_t(q) * L.C) * sizeof(T);
    }
    // the thread's own cell (a padding cell for a `pad` thread)
    __device__ T *at(int q, int dy, int dz) const {
        return (T *)(pop + row_base(q, dy, dz) + xo);
    }
    __device__ T *at_x(int q, int dy, int dz, int dx) const {
        return (T *)(pop + row_base(q, dy, dz) + xw(dx) * uint32_t(sizeof(T)));
    }
    // store addresses formed after the collision (see late_addresses)
    // (the plane stride too: otherwise the compiler keeps every plane's offset
    // from the loads live in scalar registers, and spills them, until the stores)
    __device__ void late(float after) { asm volatile("" : "+s"(pop), "+v"(xo), "+v"(x), "+s"(L.C) : "v"(after)); }
    // cell index of x + (dx, dy, dz), |d| <= 1, periodic (for per-cell arrays)
    __device__ uint32_t cell(int dx, int dy, int dz) const { return row_of(dy, dz) * nx + xw(dx); }

    // read_phase(f) runs on the complete populations inside the odd gather's
    // LDS read phase (between its barriers), where it may read other LDS arrays
    struct NoHook {
        __device__ void operator()(float (&)[M::Q]) const {}
    };
    template <int ODD, class Hook = NoHook>
    __device__ void gather(float (&f)[M::Q], T (*sh)[RB], float inv_scale, Hook &&read_phase = Hook()) const {
        if (!ODD) {
#pragma unroll
            for (int q = 0; q < M::Q; ++q) f[q] = ST::cvt(raw<T, true>(at(q, 0, 0)), inv_scale);
        } else {
            // f_q(x) = slot (opp q, x - v_q): aligned source row, x shift in LDS
            const uint32_t own = slot(0);
            int k = 0;
#pragma unroll
            for (int q = 0; q < M::Q; ++q) {
                const T v = raw<T, true>(at(M::opp(q), -M::vel(q, 1), -M::vel(q, 2)));
                if (M::vel(q, 0) == 0) f[q] = ST::cvt(v, inv_scale);
                else sh[k++][own] = v;
            }
            lds_phase_barrier();
            k = 0;
#pragma unroll
            for (int q = 0; q < M::Q; ++q)
                if (M::vel(q, 0) != 0) f[q] = ST::cvt(sh[k++][slot(-M::vel(q, 0))], inv_scale);
            read_phase(f);
            lds_phase_barrier();
        }
    }

    template <int ODD>
    __device__ void scatter(const float (&f)[M::Q], T (*sh)[RB], float scale) const {
        const bool st = live || pad;
        if (!ODD) {
            if (st) {
#pragma unroll
                for (int q = 0; q < M::Q; ++q) put<T, true>(at(M::opp(q), 0, 0), ST::pack(f[q], scale));
            }
        } else {
            // f'_q(x) goes to slot (q, x + v_q): x shift in LDS, aligned stores
            int k = 0;
#pragma unroll
            for (int q = 0; q < M::Q; ++q) {
                if (M::vel(q, 0) == 0) {
                    if (st) put<T, true>(at(q, M::vel(q, 1), M::vel(q, 2)), ST::pack(f[q], scale));
                } else {
                    sh[k++][slot(M::vel(q, 0))] = ST::pack(f[q], scale);
                }
            }
            lds_phase_barrier();
            if (st) {
                k = 0;
#pragma unroll
                for (int q = 0; q < M::Q; ++q)
                    if (M::vel(q, 0) != 0) put<T, true>(at(q, M::vel(q, 1), M::vel(q, 2)), sh[k++][x]);
            }
        }
    }

    template <int ODD>
    __device__ void gather_direct(float (&f)[M::Q], float inv_scale) const {
#pragma unroll
        for (int q = 0; q < M::Q; ++q) {
            if (!ODD) f[q] = ST::cvt(raw<T, true>(at(q, 0, 0)), inv_scale);
            else if (M::vel(q, 0) == 0)
                f[q] = ST::cvt(raw<T, true>(at(M::opp(q), -M::vel(q, 1), -M::vel(q, 2))), inv_scale);
            else
                f[q] = ST::cvt(raw<T, false>(at_x(M::opp(q), -M::vel(q, 1), -M::vel(q, 2), -M::vel(q, 0))),
                               inv_scale);
        }
    }

    template <int ODD>
    __device__ void scatter_direct(const float (&f)[M::Q], float scale) const {
        if (live) {
#pragma unroll
            for (int q = 0; q < M::Q; ++q) {
                if (!ODD) put<T, true>(at(M::opp(q), 0, 0), ST::pack(f[q], scale));
                else if (M::vel(q, 0) == 0) put<T, true>(at(q, M::vel(q, 1), M::vel(q, 2)), ST::pack(f[q], scale));
                else put<T, false>(at_x(q, M::vel(q, 1), M::vel(q, 2), M::vel(q, 0)), ST::pack(f[q], scale));
            }
        } else if (pad) {  // own padding cell, every population
#pragma unroll
            for (int q = 0; q < M::Q; ++q)
                put<T, false>(at(q, ODD ? M::vel(q, 1) : 0, ODD ? M::vel(q, 2) : 0), ST::pack(f[q], scale));
        }
    }
};

// ------------------------------------------------------------ record exchange
// Shifted storage in the row form (a block's threads on one x-row, RowIO).
// Population q arriving at x adds back phi_q of the record at x - v_q.  The
// two velocities with the same (v_y, v_z) and opposite x components read one
// neighbour row at x - 1 and x + 1.  Instead of two shifted record loads per
// cell, each thread loads that row's record at its own x (aligned), evaluates
// phi for the reader at x + 1 and for the reader at x - 1, and passes both
// through LDS (xs).  Velocities without an x component load their record at x
// directly.  The values are the ones unshift() adds, bit for bit.
template <class M>
constexpr int n_xvel() {
    int n = 0;
    for (int k = 0; k < Shift<M>::kNV; ++k) n += Shift<M>::vel(k, 0) != 0;
    return n;
}
// rank of velocity k among those with (xv = true) or without an x component
template <class M>
constexpr int vel_rank(int k, bool xv) {
    int n = 0;
    for (int j = 0; j < k; ++j) n += (Shift<M>::vel(j, 0) != 0) == xv;
    return n;
}
// the velocity with the opposite x component and the same (v_y, v_z)
template <class M>
constexpr int xvel_partner(int k) {
    for (int j = 0; j < Shift<M>::kNV; ++j)
        if (Shift<M>::vel(j, 0) == -Shift<M>::vel(k, 0) && Shift<M>::vel(j, 1) == Shift<M>::vel(k, 1) &&
            Shift<M>::vel(j, 2) == Shift<M>::vel(k, 2))
            return j;
    return -1;
}
template <class M>
constexpr bool xvel_paired() {
    for (int k = 0; k < Shift<M>::kNV; ++k)
        if (Shift<M>::vel(k, 0) != 0 && xvel_partner<M>(k) < 0) return false;
    return true;
}
static_assert(xvel_paired<MM>() && xvel_paired<MMD>() && xvel_paired<HV>(), "x velocities come in opposite pairs");

template <class M, int RB>
struct RecX {
    using S = Shift<M>;
    static constexpr int kX = n_xvel<M>(), kN = S::kNV - kX, P = S::kNPhi;
    // Worth it where most velocities have an x component (MM and the
    // difference form: 8 of 12).  HV (2 of 6, six phi values per velocity)
    // saves one record load of six and measured slower with the exchange.
    static constexpr bool kUse = 2 * kX >= S::kNV;
    // xs: LDS float[kX * P][RB]; un: phi of the velocities without an x
    // component, held from the record load until the populations are gathered
    template <int K = 0, class IO>
    __device__ static void publish(const IO &io, const u32x4 *__restrict__ rec, float (*xs)[RB],
                                   float (&un)[kN][P]) {
        if constexpr (K < S::kNV) {
            constexpr int vx = S::vel(K, 0), vy = S::vel(K, 1), vz = S::vel(K, 2);
            if constexpr (vx == 0) {
                S::template phi<K>(rec_unpack(rec[io.cell(0, -vy, -vz)]), 1.f, un[vel_rank<M>(K, false)]);
            } else if constexpr (vx > 0) {
                constexpr int K2 = xvel_partner<M>(K);
                const Rec r = rec_unpack(rec[io.cell(0, -vy, -vz)]);
                float up[P], um[P];
                S::template phi<K>(r, 1.f, up);   // for the reader at x + 1
                S::template phi<K2>(r, 1.f, um);  // for the reader at x - 1
                const uint32_t sp = io.slot(1), sm = io.slot(-1);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    xs[vel_rank<M>(K, true) * P + j][sp] = up[j];
                    xs[vel_rank<M>(K2, true) * P + j][sm] = um[j];
                }
            }
            publish<K + 1>(io, rec, xs, un);
        }
    }
    // after a barrier: add every velocity's phi to the gathered populations
    template <int K = 0, class IO>
    __device__ static void collect(const IO &io, const float (*xs)[RB], const float (&un)[kN][P],
                                   float (&f)[M::Q]) {
        if constexpr (K < S::kNV) {
            if constexpr (S::vel(K, 0) == 0) {
                S::template apply<K>(f, un[vel_rank<M>(K, false)]);
            } else {
                const uint32_t own = io.slot(0);
                float u[P];
#pragma unroll
                for (int j = 0; j < P; ++j) u[j] = xs[vel_rank<M>(K, true) * P + j][own];
                S::template apply<K>(f, u);
            }
            collect<K + 1>(io, xs, un, f);
        }
    }
};

// ------------------------------------------------------------ reductions
// Sum of one double per thread over a block of kBlock threads, in a fixed
// order (wavefront butterfly, then the NW wave partials in order).  The
// result is valid in thread 0.  `sm` is a __shared__ double[NW].
template <int NW = kBlock / 64>
__device__ __forceinline__ double block_sum(double v, double *sm) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sm[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NW; ++w) r += sm[w];
    return r;
}

}  // namespace lbem
