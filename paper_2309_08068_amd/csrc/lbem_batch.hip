// lbem_batch.hip -- many independent ragged 1-D lattices advanced by one
// persistent kernel launch (the batched form of the stepper; include/lbem.h).
//
// Every workgroup owns a list of whole instances, planned on the host longest
// first onto the least-loaded workgroup.  It advances each of its instances
// through all requested steps, one barrier per step; instances never share
// cells, so no grid-wide synchronisation exists.  The per-cell update is the
// same collision and in-place AA streaming as the 3-D kernels, restricted to
// the z component of the velocities (x and y wrap onto the cell itself).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <queue>
#include <vector>

#include "../../include/lbem.h"
#include "lbem_common.hpp"
#include "lbem_internal.hpp"
#include "lbem_util_kernels.hpp"

using namespace lbem;

namespace {

constexpr int kMaxGroups = 4096;

struct BatchArgs {
    void *pop;
    PopLayout pl;  // chunks of cells (a "row" is one cell here)
    const float *eps, *mu, *sig;
    const int32_t *inst_off;  // [n + 1]
    const int32_t *wg_start;  // [G + 1] ranges into items
    const int32_t *items;     // instance ids
    size_t total;
    int64_t nsteps;
    int32_t parity;  // time level parity at the first step
    int32_t tb_k;    // temporal blocking: steps per pass over an instance (even, <= kMaxBlockSteps)
    uint32_t pop_bytes;  // size of the population array (temporal blocking needs < 2^31)
};

constexpr int kMaxBlockSteps = 64;

// One cell of a 1-D instance occupying global cells [s, s + L).  Populations
// are in chunks of cells (PopLayout with rows of one cell): element (q, g) is
// base(g) + q * C, so a workgroup's instance spans one or two chunks.
template <class M, int ODD, class ST>
__device__ __forceinline__ void cell_1d(typename ST::T *__restrict__ pop, const PopLayout &pl, const float *eps,
                                        const float *mu, const float *sig, uint32_t s, uint32_t L, uint32_t i,
                                        CellFields *out) {
    const uint32_t g = s + i;
    const uint32_t gm = s + (i == 0 ? L - 1 : i - 1);
    const uint32_t gp = s + (i + 1 == L ? 0 : i + 1);
    const uint64_t b = pl.base(g), bm = pl.base(gm), bp = pl.base(gp);
    const uint64_t C = pl.C;
    float f[M::Q];
#pragma unroll
    for (int q = 0; q < M::Q; ++q) {
        const int vz = M::vel(q, 2);
        if (ODD) f[q] = ST::cvt(pop[uint64_t(M::opp(q)) * C + (vz > 0 ? bm : (vz < 0 ? bp : b))], 1.f);
        else f[q] = ST::cvt(pop[uint64_t(q) * C + b], 1.f);
    }
    const CellMedia m{eps[g], mu[g], sig[g]};
    const float Js[3] = {0.f, 0.f, 0.f};
    CellFields o;
    Cell<M>::collide(f, m, Js, o);
    if (out) {
        *out = o;
        return;
    }
    // store addresses formed after the collision (see late_addresses)
    uint64_t b2 = b, bm2 = bm, bp2 = bp;
    typename ST::T *pop2 = pop;
    asm volatile("" : "+v"(b2), "+v"(bm2), "+v"(bp2), "+s"(pop2) : "v"(f[0]));
#pragma unroll
    for (int q = 0; q < M::Q; ++q) {
        const int vz = M::vel(q, 2);
        if (ODD) pop2[uint64_t(q) * C + (vz > 0 ? bp2 : (vz < 0 ? bm2 : b2))] = ST::pack(f[q], 1.f);
        else pop2[uint64_t(M::opp(q)) * C + b2] = ST::pack(f[q], 1.f);
    }
}

template <class M, class ST, int T>
__global__ __launch_bounds__(T) void batch_persistent(BatchArgs a) {
    auto *pop = static_cast<typename ST::T *>(a.pop);
    const int i0 = a.wg_start[blockIdx.x], i1 = a.wg_start[blockIdx.x + 1];
    for (int it = i0; it < i1; ++it) {
        const int b = a.items[it];
        const uint32_t s = uint32_t(a.inst_off[b]);
        const uint32_t L = uint32_t(a.inst_off[b + 1]) - s;
        for (int64_t k = 0; k < a.nsteps; ++k) {
            if (((a.parity + k) & 1) == 0) {
                for (uint32_t i = threadIdx.x; i < L; i += T)
                    cell_1d<M, 0, ST>(pop, a.pl, a.eps, a.mu, a.sig, s, L, i, nullptr);
            } else {
                for (uint32_t i = threadIdx.x; i < L; i += T)
                    cell_1d<M, 1, ST>(pop, a.pl, a.eps, a.mu, a.sig, s, L, i, nullptr);
            }
            lds_phase_barrier();  // the next step reads what neighbouring threads wrote
        }
    }
}

// ---------------------------------------------------------------- temporal blocking
// Slot of population q among the populations of M with the same z velocity
// (the LDS exchange arrays hold only the populations that move in 1-D).
template <class M>
__host__ __device__ constexpr int zslot(int q) {
    int n = 0;
    for (int p = 0; p < q; ++p)
        if (M::vel(p, 2) == M::vel(q, 2)) ++n;
    return n;
}
template <class M>
__host__ __device__ constexpr int zcount(int sgn) {
    int n = 0;
    for (int q = 0; q < M::Q; ++q)
        if (M::vel(q, 2) == sgn) ++n;
    return n;
}

// One step of the cell a thread holds in registers: collision, the storage
// format's rounding of every post-collision value (as the one-step schedule
// stores and reloads them, so both schedules give the same bits), then
// streaming through LDS: +z movers arrive from thread `left`, -z movers from
// thread `right`.  With NB = 2, xch is one of two alternating buffers and one
// barrier per step suffices: a thread can only overwrite a buffer after every
// thread has passed the barrier that follows its reads of that buffer.  With
// NB = 1 (1024 threads, where two buffers do not fit in LDS) a second
// barrier separates the reads from the next step's writes.
template <class M, class ST, int T, int NB>
__device__ __forceinline__ void tb_step(float (&f)[M::Q], const CellMedia &m, float *xch, uint32_t tid, uint32_t left,
                                        uint32_t right) {
    constexpr int NP = zcount<M>(1);
    const float Js[3] = {0.f, 0.f, 0.f};
    CellFields o;
    Cell<M>::collide(f, m, Js, o);
#pragma unroll
    for (int q = 0; q < M::Q; ++q) {
        f[q] = ST::cvt(ST::pack(f[q], 1.f), 1.f);
        const int vz = M::vel(q, 2);
        if (vz > 0) xch[zslot<M>(q) * T + tid] = f[q];
        if (vz < 0) xch[(NP + zslot<M>(q)) * T + tid] = f[q];
    }
    lds_phase_barrier();
#pragma unroll
    for (int q = 0; q < M::Q; ++q) {
        const int vz = M::vel(q, 2);
        if (vz > 0) f[q] = xch[zslot<M>(q) * T + left];
        if (vz < 0) f[q] = xch[(NP + zslot<M>(q)) * T + right];
    }
    if constexpr (NB == 1) lds_phase_barrier();
}

// Population access of the temporally blocked kernel through a buffer
// resource: a per-thread byte offset (the cell) plus a uniform byte offset (the
// population plane) held in a scalar register, so Q loads in flight cost no
// address registers.  The hardware checks every offset against the array size.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(void *pop, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(pop, 0, int(bytes), 0x00020000);  // raw dwords, gfx9 word 3
}
template <class ST>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(typename ST::T) == 4)
        return ST::cvt(__builtin_bit_cast(typename ST::T, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0)), 1.f);
    else
        return ST::cvt(__builtin_bit_cast(typename ST::T, __builtin_amdgcn_raw_buffer_load_b16(r, int(voff), int(soff), 0)), 1.f);
}
template <class ST>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    if constexpr (sizeof(typename ST::T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, ST::pack(v, 1.f)), r, int(voff), int(soff), 0);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, ST::pack(v, 1.f)), r, int(voff), int(soff), 0);
}

// Temporally blocked form of batch_persistent.  Each pass advances an
// instance by k steps (k even) with the cells held in registers:
//   - L <= T: the whole instance is resident (thread i holds cell i, periodic
//     neighbours) and one pass covers every even step of the call;
//   - L > T: trapezoidal tiles of T cells, each computing the T - 2k cells
//     it can update exactly (information moves one cell per step) and
//     storing them in place; the halo cells a later tile needs at the old
//     time level (the k cells left of its interior, overwritten by the tile
//     before, and cells 0..k-1 where a right halo wraps past the end of the
//     instance, overwritten by the first tile) are kept in LDS.
// Between passes the state is at an even time level, where population q of
// cell g sits in slot (q, g); an odd first or last step uses the one-step code.
template <class M, class ST, int T>
__global__ __launch_bounds__(T) void batch_tb(BatchArgs a) {
    constexpr int Q = M::Q;
    constexpr int NX = zcount<M>(1) + zcount<M>(-1);
    constexpr int NB = T >= 1024 ? 1 : 2;
    __shared__ float xch[NB][NX * T];
    __shared__ float stash_left[kMaxBlockSteps * Q];
    __shared__ float stash_right[kMaxBlockSteps * Q];
    auto *pop = static_cast<typename ST::T *>(a.pop);
    const uint32_t tid = threadIdx.x;
    const uint32_t k_max = uint32_t(max(2, min(a.tb_k, kMaxBlockSteps))) & ~1u;
    constexpr uint32_t S = sizeof(typename ST::T);
    const uint32_t plane = a.pl.C * S;  // bytes between population planes of a chunk
    const __amdgpu_buffer_rsrc_t rsrc = pop_rsrc(a.pop, a.pop_bytes);
    const int i0 = a.wg_start[blockIdx.x], i1 = a.wg_start[blockIdx.x + 1];
    for (int it = i0; it < i1; ++it) {
        const int b = a.items[it];
        const uint32_t s = uint32_t(a.inst_off[b]);
        const uint32_t L = uint32_t(a.inst_off[b + 1]) - s;
        int64_t rem = a.nsteps;
        if (rem > 0 && (a.parity & 1)) {
            for (uint32_t i = tid; i < L; i += T) cell_1d<M, 1, ST>(pop, a.pl, a.eps, a.mu, a.sig, s, L, i, nullptr);
            lds_phase_barrier();
            --rem;
        }
        uint32_t sw = 0;  // exchange buffer of the next step
        while (rem >= 2) {
            float f[Q];
            if (L <= uint32_t(T)) {
                const int64_t k = rem & ~int64_t(1);
                const uint32_t c = tid < L ? tid : 0;
                const uint32_t off = uint32_t(a.pl.base(s + c)) * S;
#pragma unroll
                for (int q = 0; q < Q; ++q) f[q] = buf_ld<ST>(rsrc, off, q * plane);
                const CellMedia m{a.eps[s + c], a.mu[s + c], a.sig[s + c]};
                const uint32_t left = tid < L ? (tid == 0 ? L - 1 : tid - 1) : tid;
                const uint32_t right = tid < L ? (tid + 1 == L ? 0 : tid + 1) : tid;
                for (int64_t n = 0; n < k; ++n, sw ^= NB - 1u) tb_step<M, ST, T, NB>(f, m, xch[sw], tid, left, right);
                if (tid < L) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) buf_st<ST>(rsrc, off, q * plane, f[q]);
                }
                lds_phase_barrier();
                rem -= k;
                continue;
            }
            const uint32_t k = uint32_t(rem < int64_t(k_max) ? rem & ~int64_t(1) : int64_t(k_max));
            const uint32_t W = uint32_t(T) - 2 * k;  // cells a tile updates
            const uint32_t ntile = (L + W - 1) / W;
            for (uint32_t j = 0; j < ntile; ++j) {
                const uint32_t start = j * W;
                // cell of this thread: start - k + tid, wrapped into [0, L)
                int64_t raw = int64_t(start) - k + tid;
                const bool wrapped_right = raw >= int64_t(L);
                const uint32_t c = uint32_t(raw < 0 ? raw + L : (wrapped_right ? raw - L : raw));
                const uint32_t off = uint32_t(a.pl.base(s + c)) * S;
                // every load is issued unconditionally (all addresses are cells of the
                // instance), so the Q loads are in flight together; the halo cells an
                // earlier tile has overwritten then take their old values from LDS
#pragma unroll
                for (int q = 0; q < Q; ++q) f[q] = buf_ld<ST>(rsrc, off, q * plane);
                const CellMedia m{a.eps[s + c], a.mu[s + c], a.sig[s + c]};
                if (j > 0 && tid < k) {  // overwritten by tile j - 1
#pragma unroll
                    for (int q = 0; q < Q; ++q) f[q] = stash_left[tid * Q + q];
                }
                if (wrapped_right && c < k) {  // overwritten by tile 0
#pragma unroll
                    for (int q = 0; q < Q; ++q) f[q] = stash_right[c * Q + q];
                }
                lds_phase_barrier();  // stash reads done before the stash is rewritten
                if (j + 1 < ntile && tid >= W && tid < W + k) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) stash_left[(tid - W) * Q + q] = f[q];
                }
                if (j == 0 && tid >= k && tid < 2 * k) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) stash_right[(tid - k) * Q + q] = f[q];
                }
                const uint32_t left = tid == 0 ? 0 : tid - 1;  // edge threads read garbage that never
                const uint32_t right = tid + 1 == uint32_t(T) ? tid : tid + 1;  // reaches the interior
                for (uint32_t n = 0; n < k; ++n, sw ^= NB - 1u) tb_step<M, ST, T, NB>(f, m, xch[sw], tid, left, right);
                const uint32_t w = min(W, L - start);
                if (tid >= k && tid < k + w) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) buf_st<ST>(rsrc, off, q * plane, f[q]);
                }
                lds_phase_barrier();
            }
            rem -= k;
        }
        if (rem == 1) {
            for (uint32_t i = tid; i < L; i += T) cell_1d<M, 0, ST>(pop, a.pl, a.eps, a.mu, a.sig, s, L, i, nullptr);
            lds_phase_barrier();
        }
    }
}

// One step of one instance (the per-instance reference schedule).
template <class M, int ODD, class ST>
__global__ __launch_bounds__(kBlock) void batch_one(BatchArgs a, uint32_t s, uint32_t L) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < L) cell_1d<M, ODD, ST>(static_cast<typename ST::T *>(a.pop), a.pl, a.eps, a.mu, a.sig, s, L, i, nullptr);
}

template <class M, int ODD, class ST>
__global__ __launch_bounds__(kBlock) void batch_fields(BatchArgs a, const int32_t *cell_inst, float *E, float *B) {
    const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= a.total) return;
    const int b = cell_inst[g];
    const uint32_t s = uint32_t(a.inst_off[b]);
    const uint32_t L = uint32_t(a.inst_off[b + 1]) - s;
    CellFields o;
    cell_1d<M, ODD, ST>(static_cast<typename ST::T *>(a.pop), a.pl, a.eps, a.mu, a.sig, s, L, g - s, &o);
    for (int d = 0; d < 3; ++d) {
        if (E) E[d * a.total + g] = o.E[d];
        if (B) B[d * a.total + g] = o.B[d];
    }
}

template <class M, class ST>
__global__ __launch_bounds__(kBlock) void batch_init(void *pop, PopLayout pl, const float *eps, const float *mu,
                                                     const float *E, const float *B, uint32_t total) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= total) return;
    const CellMedia m{eps[c], mu[c], 0.f};
    const float e[3] = {E[c], E[size_t(total) + c], E[2 * size_t(total) + c]};
    const float b[3] = {B[c], B[size_t(total) + c], B[2 * size_t(total) + c]};
    float f[M::Q];
    Cell<M>::equilibrium(f, m, e, b);
    auto *p = static_cast<typename ST::T *>(pop) + pl.base(c);
#pragma unroll
    for (int q = 0; q < M::Q; ++q) p[uint64_t(q) * pl.C] = ST::pack(f[q], 1.f);
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct BatchLayout {
    size_t pop, backup, eps, mu, sig, inst_off, cell_inst, wg_start, items, flags, total;
};

// Chunks of cells with at most kChunkBytes per population plane (as for the
// 3-D lattice; a row of the layout is one cell); one chunk if all cells fit.
PopLayout batch_pop_layout(int model, int storage, size_t total) {
    const uint32_t Q = uint32_t(model_pops(model));
    const uint32_t cells = kChunkBytes / (storage == LBEM_F32 ? 4u : 2u);
    PopLayout pl{1u, 31u, uint32_t(total), 0, 1u};
    if (total > cells) {
        uint32_t sh = 0;
        while ((2u << sh) <= cells) ++sh;
        pl.rshift = sh;
        pl.C = 1u << sh;
    }
    pl.QC = uint64_t(Q) * pl.C;
    return pl;
}

BatchLayout batch_layout(int model, int storage, int32_t n, size_t total) {
    BatchLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = al(off + bytes);
        return o;
    };
    const PopLayout pl = batch_pop_layout(model, storage, total);
    const size_t nchunks = pl.rshift == 31 ? 1 : (total + pl.C - 1) / pl.C;
    const size_t pb = nchunks * pl.QC * (storage == LBEM_F32 ? 4 : 2);
    L.pop = take(pb);
    L.backup = take(pb);
    L.eps = take(total * 4);
    L.mu = take(total * 4);
    L.sig = take(total * 4);
    L.inst_off = take((size_t(n) + 1) * 4);
    L.cell_inst = take(total * 4);
    L.wg_start = take((size_t(kMaxGroups) + 1) * 4);
    L.items = take(size_t(n) * 4);
    L.flags = take(64);
    L.total = off;
    return L;
}

lbem_status check_offsets(int32_t model, int32_t storage, int32_t n, const int64_t *offsets) {
    if (model_pops(model) == 0) return fail(LBEM_EINVAL, "unknown model %d", model);
    if (storage < LBEM_F32 || storage > LBEM_F16)
        return fail(LBEM_EINVAL, "storage %d is not available for batches (plain FP32, BF16 or FP16 only)", storage);
    if (n < 1) return fail(LBEM_EINVAL, "need at least one instance");
    if (!offsets) return fail(LBEM_EINVAL, "offsets is NULL");
    if (offsets[0] != 0) return fail(LBEM_EINVAL, "offsets[0] must be 0");
    for (int32_t b = 0; b < n; ++b)
        if (offsets[b + 1] <= offsets[b]) return fail(LBEM_EINVAL, "instance %d is empty or offsets decrease", b);
    if (offsets[n] >= (int64_t(1) << 31)) return fail(LBEM_EINVAL, "total cells must be < 2^31");
    return LBEM_OK;
}

}  // namespace

struct lbem_batch {
    int model, storage;
    int32_t n;
    uint32_t total;
    std::vector<int64_t> off;
    hipStream_t stream;
    char *ws;
    BatchLayout L;
    PopLayout pl;
    int ncu;
    int threads, gpc, groups;
    int tb_k;  // steps per temporally blocked pass, 0 = one step per pass
    int64_t t;
    // cached graph of one persistent launch
    hipGraphExec_t gexec;
    hipGraph_t graph;
    int64_t g_nsteps;
    int g_parity;
    int g_threads, g_gpc, g_tb;
};

namespace {

template <class T>
T *at(lbem_batch *b, size_t off) {
    return reinterpret_cast<T *>(b->ws + off);
}

BatchArgs args_of(lbem_batch *b, int64_t nsteps) {
    BatchArgs a{};
    a.pop = b->ws + b->L.pop;
    a.pl = b->pl;
    a.eps = at<const float>(b, b->L.eps);
    a.mu = at<const float>(b, b->L.mu);
    a.sig = at<const float>(b, b->L.sig);
    a.inst_off = at<const int32_t>(b, b->L.inst_off);
    a.wg_start = at<const int32_t>(b, b->L.wg_start);
    a.items = at<const int32_t>(b, b->L.items);
    a.total = b->total;
    a.nsteps = nsteps;
    a.parity = int32_t(b->t & 1);
    a.tb_k = b->tb_k;
    a.pop_bytes = uint32_t(std::min<size_t>(b->L.backup - b->L.pop, 0xffffffffu));
    return a;
}

// Longest-processing-time-first plan of instances onto `groups` workgroups.
lbem_status plan(lbem_batch *b) {
    const int G = b->groups;
    std::vector<int32_t> order(b->n);
    for (int32_t i = 0; i < b->n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        const int64_t lx = b->off[x + 1] - b->off[x], ly = b->off[y + 1] - b->off[y];
        return lx != ly ? lx > ly : x < y;
    });
    using Bin = std::pair<int64_t, int>;  // (load, group)
    std::priority_queue<Bin, std::vector<Bin>, std::greater<Bin>> heap;
    for (int g = 0; g < G; ++g) heap.push({0, g});
    std::vector<std::vector<int32_t>> bins(G);
    for (int32_t i : order) {
        Bin top = heap.top();
        heap.pop();
        bins[top.second].push_back(i);
        top.first += b->off[i + 1] - b->off[i];
        heap.push(top);
    }
    std::vector<int32_t> start(G + 1), items;
    items.reserve(b->n);
    for (int g = 0; g < G; ++g) {
        start[g] = int32_t(items.size());
        items.insert(items.end(), bins[g].begin(), bins[g].end());
    }
    start[G] = int32_t(items.size());
    lbem_status st = hip_check(hipMemcpyAsync(b->ws + b->L.wg_start, start.data(), start.size() * 4,
                                              hipMemcpyHostToDevice, b->stream), "copy plan");
    if (!st) st = hip_check(hipMemcpyAsync(b->ws + b->L.items, items.data(), items.size() * 4, hipMemcpyHostToDevice,
                                           b->stream), "copy plan");
    if (!st) st = hip_check(hipStreamSynchronize(b->stream), "synchronise");
    return st;
}

template <class M, class ST>
void launch_persistent_t(lbem_batch *b, const BatchArgs &a, hipStream_t s) {
    if (b->tb_k > 0) {
        if (b->threads == 256) hipLaunchKernelGGL((batch_tb<M, ST, 256>), dim3(b->groups), dim3(256), 0, s, a);
        else if (b->threads == 512) hipLaunchKernelGGL((batch_tb<M, ST, 512>), dim3(b->groups), dim3(512), 0, s, a);
        else hipLaunchKernelGGL((batch_tb<M, ST, 1024>), dim3(b->groups), dim3(1024), 0, s, a);
        return;
    }
    switch (b->threads) {
        case 128: hipLaunchKernelGGL((batch_persistent<M, ST, 128>), dim3(b->groups), dim3(128), 0, s, a); break;
        case 256: hipLaunchKernelGGL((batch_persistent<M, ST, 256>), dim3(b->groups), dim3(256), 0, s, a); break;
        case 512: hipLaunchKernelGGL((batch_persistent<M, ST, 512>), dim3(b->groups), dim3(512), 0, s, a); break;
        default: hipLaunchKernelGGL((batch_persistent<M, ST, 1024>), dim3(b->groups), dim3(1024), 0, s, a); break;
    }
}

template <class M>
void launch_persistent_m(lbem_batch *b, const BatchArgs &a, hipStream_t s) {
    switch (b->storage) {
        case LBEM_F32: launch_persistent_t<M, StF32>(b, a, s); break;
        case LBEM_BF16: launch_persistent_t<M, StBF16>(b, a, s); break;
        default: launch_persistent_t<M, StF16>(b, a, s); break;
    }
}

void launch_persistent(lbem_batch *b, int64_t nsteps, hipStream_t s) {
    const BatchArgs a = args_of(b, nsteps);
    if (b->model == LBEM_MM) launch_persistent_m<MM>(b, a, s);
    else if (b->model == LBEM_MM_DIFF) launch_persistent_m<MMD>(b, a, s);
    else launch_persistent_m<HV>(b, a, s);
}

template <class M, int ODD, class ST>
void launch_one(const BatchArgs &a, uint32_t s0, uint32_t L, hipStream_t s) {
    hipLaunchKernelGGL((batch_one<M, ODD, ST>), dim3((L + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a, s0, L);
}

template <class M, int ODD>
void launch_one_st(lbem_batch *b, const BatchArgs &a, uint32_t s0, uint32_t L) {
    switch (b->storage) {
        case LBEM_F32: launch_one<M, ODD, StF32>(a, s0, L, b->stream); break;
        case LBEM_BF16: launch_one<M, ODD, StBF16>(a, s0, L, b->stream); break;
        default: launch_one<M, ODD, StF16>(a, s0, L, b->stream); break;
    }
}

template <class M, int ODD, class ST>
void launch_fields(lbem_batch *b, const BatchArgs &a, float *E, float *B) {
    hipLaunchKernelGGL((batch_fields<M, ODD, ST>), dim3((b->total + kBlock - 1) / kBlock), dim3(kBlock), 0, b->stream,
                       a, at<const int32_t>(b, b->L.cell_inst), E, B);
}

template <class M, int ODD>
void launch_fields_st(lbem_batch *b, const BatchArgs &a, float *E, float *B) {
    switch (b->storage) {
        case LBEM_F32: launch_fields<M, ODD, StF32>(b, a, E, B); break;
        case LBEM_BF16: launch_fields<M, ODD, StBF16>(b, a, E, B); break;
        default: launch_fields<M, ODD, StF16>(b, a, E, B); break;
    }
}

void drop_graph(lbem_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

}  // namespace

lbem_status lbem_batch_workspace_size(int32_t model, int32_t storage, int32_t n, const int64_t *offsets,
                                      size_t *bytes) {
    lbem_status st = check_offsets(model, storage, n, offsets);
    if (st) return st;
    if (!bytes) return fail(LBEM_EINVAL, "bytes is NULL");
    *bytes = batch_layout(model, storage, n, size_t(offsets[n])).total;
    return LBEM_OK;
}

lbem_status lbem_batch_create(int32_t model, int32_t storage, int32_t n, const int64_t *offsets, const float *eps_r,
                              const float *mu_r, const float *sigma, void *workspace, size_t workspace_bytes,
                              void *stream, lbem_batch **out) {
    lbem_status st = check_offsets(model, storage, n, offsets);
    if (st) return st;
    if (!out || !workspace) return fail(LBEM_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(LBEM_EINVAL, "workspace must be 256-byte aligned");
    const size_t total = size_t(offsets[n]);
    const BatchLayout L = batch_layout(model, storage, n, total);
    if (workspace_bytes < L.total) return fail(LBEM_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    int dev = 0, ncu = 0;
    st = hip_check(hipGetDevice(&dev), "get device");
    if (!st) st = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
    if (st) return st;
    auto *b = new (std::nothrow) lbem_batch();
    if (!b) return fail(LBEM_ENOMEM, "host allocation failed");
    b->model = model;
    b->storage = storage;
    b->n = n;
    b->total = uint32_t(total);
    b->off.assign(offsets, offsets + n + 1);
    b->stream = static_cast<hipStream_t>(stream);
    b->ws = static_cast<char *>(workspace);
    b->L = L;
    b->pl = batch_pop_layout(model, storage, total);
    b->ncu = ncu > 0 ? ncu : 1;
    b->threads = 256;
    b->gpc = 2;
    b->groups = std::min(kMaxGroups, b->ncu * b->gpc);
    hipStream_t s = b->stream;
    const uint32_t g = uint32_t((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(fill_or_copy, dim3(g), dim3(kBlock), 0, s, at<float>(b, L.eps), eps_r, 1.0f, b->total);
    hipLaunchKernelGGL(fill_or_copy, dim3(g), dim3(kBlock), 0, s, at<float>(b, L.mu), mu_r, 1.0f, b->total);
    hipLaunchKernelGGL(fill_or_copy, dim3(g), dim3(kBlock), 0, s, at<float>(b, L.sig), sigma, 0.0f, b->total);
    const size_t popw = (L.backup - L.pop) / 4;
    hipLaunchKernelGGL(zero_bytes, dim3(uint32_t((popw + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       at<uint32_t>(b, L.pop), popw);
    hipLaunchKernelGGL(zero_bytes, dim3(1), dim3(kBlock), 0, s, at<uint32_t>(b, L.flags), size_t(16));
    std::vector<int32_t> off32(n + 1), cell_inst(total);
    for (int32_t i = 0; i <= n; ++i) off32[i] = int32_t(offsets[i]);
    for (int32_t i = 0; i < n; ++i)
        std::fill(cell_inst.begin() + offsets[i], cell_inst.begin() + offsets[i + 1], i);
    int32_t counts[4] = {0, 0, 0, 0};
    hipLaunchKernelGGL(validate_media, dim3(g), dim3(kBlock), 0, s, at<const float>(b, L.eps), at<const float>(b, L.mu),
                       at<const float>(b, L.sig), b->total, model, at<int32_t>(b, L.flags));
    st = hip_check(hipGetLastError(), "launch");
    if (!st) st = hip_check(hipMemcpyAsync(b->ws + L.inst_off, off32.data(), off32.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipMemcpyAsync(b->ws + L.cell_inst, cell_inst.data(), cell_inst.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (!st) st = hip_check(hipMemcpyAsync(counts, b->ws + L.flags, sizeof(counts), hipMemcpyDeviceToHost, s), "copy flags");
    if (!st) st = hip_check(hipStreamSynchronize(s), "synchronise");
    if (!st && counts[0]) st = fail(LBEM_ENOTFINITE, "%d cells have non-finite media", counts[0]);
    if (!st && counts[1]) st = fail(LBEM_EINVAL, "%d cells have eps_r <= 0, mu_r <= 0 or sigma < 0", counts[1]);
    if (!st && counts[2]) st = fail(LBEM_EUNSTABLE, "%d cells have eps_r * mu_r < 1", counts[2]);
    if (!st && counts[3]) st = fail(LBEM_EUNSTABLE, "%d cells have sigma / (3 eps_r) >= 2 (HV current)", counts[3]);
    if (!st) st = plan(b);
    if (st) {
        delete b;
        return st;
    }
    *out = b;
    return LBEM_OK;
}

lbem_status lbem_batch_destroy(lbem_batch *b) {
    if (!b) return fail(LBEM_EINVAL, "batch is NULL");
    drop_graph(b);
    delete b;
    return LBEM_OK;
}

template <class M>
static void batch_init_m(lbem_batch *b, const float *E, const float *B) {
    const uint32_t g = (b->total + kBlock - 1) / kBlock;
    void *pop = b->ws + b->L.pop;
    const float *eps = at<const float>(b, b->L.eps), *mu = at<const float>(b, b->L.mu);
    switch (b->storage) {
        case LBEM_F32: hipLaunchKernelGGL((batch_init<M, StF32>), dim3(g), dim3(kBlock), 0, b->stream, pop, b->pl, eps, mu, E, B, b->total); break;
        case LBEM_BF16: hipLaunchKernelGGL((batch_init<M, StBF16>), dim3(g), dim3(kBlock), 0, b->stream, pop, b->pl, eps, mu, E, B, b->total); break;
        default: hipLaunchKernelGGL((batch_init<M, StF16>), dim3(g), dim3(kBlock), 0, b->stream, pop, b->pl, eps, mu, E, B, b->total); break;
    }
}

lbem_status lbem_batch_set_fields(lbem_batch *b, const float *E, const float *B) {
    if (!b || !E || !B) return fail(LBEM_EINVAL, "null argument");
    if (b->model == LBEM_MM) batch_init_m<MM>(b, E, B);
    else if (b->model == LBEM_MM_DIFF) batch_init_m<MMD>(b, E, B);
    else batch_init_m<HV>(b, E, B);
    b->t = 0;
    return hip_check(hipGetLastError(), "init launch");
}

lbem_status lbem_batch_set_launch(lbem_batch *b, int32_t threads, int32_t groups_per_cu) {
    if (!b) return fail(LBEM_EINVAL, "batch is NULL");
    if (threads != 128 && threads != 256 && threads != 512 && threads != 1024)
        return fail(LBEM_EINVAL, "threads must be 128, 256, 512 or 1024");
    if (b->tb_k > 0 && threads < 256)
        return fail(LBEM_EINVAL, "temporal blocking runs 256, 512 or 1024 threads per workgroup");
    if (groups_per_cu < 1 || int64_t(groups_per_cu) * b->ncu > kMaxGroups)
        return fail(LBEM_EINVAL, "groups_per_cu must be in [1, %d]", kMaxGroups / b->ncu);
    b->threads = threads;
    b->gpc = groups_per_cu;
    b->groups = b->ncu * groups_per_cu;
    return plan(b);
}

lbem_status lbem_batch_set_blocking(lbem_batch *b, int32_t steps_per_pass) {
    if (!b) return fail(LBEM_EINVAL, "batch is NULL");
    if (steps_per_pass != 0 &&
        (steps_per_pass < 2 || steps_per_pass > kMaxBlockSteps || (steps_per_pass & 1)))
        return fail(LBEM_EINVAL, "steps_per_pass must be 0 or even in [2, %d]", kMaxBlockSteps);
    if (steps_per_pass > 0 && b->threads < 256)
        return fail(LBEM_EINVAL, "temporal blocking runs 256, 512 or 1024 threads per workgroup (see lbem_batch_set_launch)");
    if (steps_per_pass > 0 && b->L.backup - b->L.pop >= (size_t(1) << 31))
        return fail(LBEM_EINVAL, "temporal blocking needs a population array below 2 GiB (this batch has %zu bytes)",
                    b->L.backup - b->L.pop);
    b->tb_k = steps_per_pass;
    return LBEM_OK;
}

lbem_status lbem_batch_get_blocking(lbem_batch *b, int32_t *steps_per_pass) {
    if (!b || !steps_per_pass) return fail(LBEM_EINVAL, "null argument");
    *steps_per_pass = b->tb_k;
    return LBEM_OK;
}

lbem_status lbem_batch_step(lbem_batch *b, int64_t nsteps) {
    if (!b) return fail(LBEM_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(LBEM_EINVAL, "nsteps < 0");
    if (nsteps == 0) return LBEM_OK;
    launch_persistent(b, nsteps, b->stream);
    lbem_status st = hip_check(hipGetLastError(), "persistent launch");
    if (!st) b->t += nsteps;
    return st;
}

lbem_status lbem_batch_step_graph(lbem_batch *b, int64_t nsteps) {
    if (!b) return fail(LBEM_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(LBEM_EINVAL, "nsteps < 0");
    if (nsteps == 0) return LBEM_OK;
    const int parity = int(b->t & 1);
    if (!b->gexec || b->g_nsteps != nsteps || b->g_parity != parity || b->g_threads != b->threads ||
        b->g_gpc != b->gpc || b->g_tb != b->tb_k) {
        drop_graph(b);
        // capture on a private stream (the null stream cannot be captured)
        hipStream_t cs = nullptr;
        lbem_status st = hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
        if (st) return st;
        st = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
        if (!st) {
            launch_persistent(b, nsteps, cs);
            hipGraph_t g = nullptr;
            st = hip_check(hipStreamEndCapture(cs, &g), "end capture");
            if (!st) {
                b->graph = g;
                st = hip_check(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0), "instantiate graph");
            }
        }
        (void)hipStreamDestroy(cs);
        if (st) {
            drop_graph(b);
            return st;
        }
        b->g_nsteps = nsteps;
        b->g_parity = parity;
        b->g_threads = b->threads;
        b->g_gpc = b->gpc;
        b->g_tb = b->tb_k;
    }
    lbem_status st = hip_check(hipGraphLaunch(b->gexec, b->stream), "graph launch");
    if (!st) b->t += nsteps;
    return st;
}

lbem_status lbem_batch_step_per_instance(lbem_batch *b, int64_t nsteps) {
    if (!b) return fail(LBEM_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(LBEM_EINVAL, "nsteps < 0");
    for (int64_t k = 0; k < nsteps; ++k) {
        const BatchArgs a = args_of(b, 1);
        const int odd = int(b->t & 1);
        for (int32_t i = 0; i < b->n; ++i) {
            const uint32_t s0 = uint32_t(b->off[i]), L = uint32_t(b->off[i + 1] - b->off[i]);
            if (b->model == LBEM_MM) {
                if (odd) launch_one_st<MM, 1>(b, a, s0, L);
                else launch_one_st<MM, 0>(b, a, s0, L);
            } else if (b->model == LBEM_MM_DIFF) {
                if (odd) launch_one_st<MMD, 1>(b, a, s0, L);
                else launch_one_st<MMD, 0>(b, a, s0, L);
            } else {
                if (odd) launch_one_st<HV, 1>(b, a, s0, L);
                else launch_one_st<HV, 0>(b, a, s0, L);
            }
        }
        lbem_status st = hip_check(hipGetLastError(), "per-instance launch");
        if (st) return st;
        b->t += 1;
    }
    return LBEM_OK;
}

lbem_status lbem_batch_get_fields(lbem_batch *b, float *E, float *B) {
    if (!b) return fail(LBEM_EINVAL, "batch is NULL");
    const BatchArgs a = args_of(b, 0);
    const int odd = int(b->t & 1);
    if (b->model == LBEM_MM) {
        if (odd) launch_fields_st<MM, 1>(b, a, E, B);
        else launch_fields_st<MM, 0>(b, a, E, B);
    } else if (b->model == LBEM_MM_DIFF) {
        if (odd) launch_fields_st<MMD, 1>(b, a, E, B);
        else launch_fields_st<MMD, 0>(b, a, E, B);
    } else {
        if (odd) launch_fields_st<HV, 1>(b, a, E, B);
        else launch_fields_st<HV, 0>(b, a, E, B);
    }
    return hip_check(hipGetLastError(), "fields launch");
}

lbem_status lbem_batch_get_time(lbem_batch *b, int64_t *t) {
    if (!b || !t) return fail(LBEM_EINVAL, "null argument");
    *t = b->t;
    return LBEM_OK;
}

lbem_status lbem_batch_autotune(lbem_batch *b, int32_t trial_steps, int32_t *threads, int32_t *groups_per_cu) {
    if (!b) return fail(LBEM_EINVAL, "batch is NULL");
    if (trial_steps < 1) return fail(LBEM_EINVAL, "trial_steps must be >= 1");
    // (threads, groups per CU, steps per temporally blocked pass)
    static const int32_t cand[][3] = {{256, 1, 0},  {256, 2, 0},  {256, 4, 0},  {512, 1, 0},  {512, 2, 0},
                                      {1024, 1, 0}, {128, 4, 0},  {128, 8, 0},  {256, 2, 16}, {256, 2, 32},
                                      {512, 1, 16}, {512, 1, 32}, {512, 1, 48}, {512, 2, 32}, {1024, 1, 32},
                                      {1024, 1, 48}, {1024, 1, 64}};
    const size_t pb = b->L.backup - b->L.pop;
    const int64_t t_saved = b->t;
    lbem_status st = hip_check(hipMemcpyAsync(b->ws + b->L.backup, b->ws + b->L.pop, pb, hipMemcpyDeviceToDevice, b->stream), "backup");
    if (st) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    st = hip_check(hipEventCreate(&e0), "event");
    if (!st) st = hip_check(hipEventCreate(&e1), "event");
    float best = 1e30f;
    int32_t bt = b->threads, bg = b->gpc, bk = b->tb_k;
    for (const auto &c : cand) {
        if (st) break;
        if (int64_t(c[1]) * b->ncu > kMaxGroups) continue;
        if (c[2] > 0 && b->L.backup - b->L.pop >= (size_t(1) << 31)) continue;
        b->tb_k = 0;
        st = lbem_batch_set_launch(b, c[0], c[1]);
        if (!st) st = lbem_batch_set_blocking(b, c[2]);
        if (st) break;
        // a blocked candidate is timed over at least two full passes
        const int64_t steps = std::max<int64_t>(trial_steps, 2 * c[2]);
        launch_persistent(b, 2, b->stream);  // warm-up
        st = hip_check(hipEventRecord(e0, b->stream), "record");
        if (!st) launch_persistent(b, steps, b->stream);
        if (!st) st = hip_check(hipEventRecord(e1, b->stream), "record");
        if (!st) st = hip_check(hipEventSynchronize(e1), "sync");
        float ms = 0.f;
        if (!st) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        if (!st) ms /= float(steps);
        if (!st && ms < best) {
            best = ms;
            bt = c[0];
            bg = c[1];
            bk = c[2];
        }
        // restore the state for the next candidate
        if (!st) st = hip_check(hipMemcpyAsync(b->ws + b->L.pop, b->ws + b->L.backup, pb, hipMemcpyDeviceToDevice, b->stream), "restore");
        b->t = t_saved;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) return st;
    b->tb_k = 0;
    st = lbem_batch_set_launch(b, bt, bg);
    if (!st) st = lbem_batch_set_blocking(b, bk);
    if (st) return st;
    if (threads) *threads = bt;
    if (groups_per_cu) *groups_per_cu = bg;
    return LBEM_OK;
}
