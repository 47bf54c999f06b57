// lbem_adjoint.hip -- reverse-time (adjoint) differentiation of the
// detector-plane loss with respect to the per-cell eps_r and sigma (MM model).
//
// Forward, for fixed media theta = (eps_r, sigma):  f_{n+1} = S C_theta f_n,
// with C(f) = 2 f_eq(m(f); theta) - f (Section II) and S the advection.
// Loss L = sum_n l(f_n), l(f) = sum over the plane z_d of |E(f)|^2.
// Adjoint:   mu_n = S^T lambda_{n+1},   lambda_n = C_theta^T mu_n + dl/df_n,
//            lambda_{t0+N} = 0,
// gradient:  dL/dtheta_x += 2 mu_n(x) . d f_eq(E_n(x); theta_x) / dtheta_x
//                           + dl(f_n)/dtheta_x  [+ lambda_0 . df_0/dtheta at t0].
// S^T is streaming with reversed velocities, so the adjoint step is the same
// in-place AA gather / scatter with v -> -v.  C^T is rank-structured:
// C^T mu = 2 M^T U^T mu - mu, with U^T mu a handful of adjoint moments and
// M^T distributing them back, at the cost of one forward collision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/lbem.h"
#include "lbem_common.hpp"
#include "lbem_internal.hpp"
#include "lbem_util_kernels.hpp"

using namespace lbem;

namespace {

// MM with every velocity reversed: the AA streaming of S^T.
struct MMRev {
    static constexpr int Q = 50;
    __host__ __device__ static constexpr int vel(int q, int a) { return -MM::vel(q, a); }
    __host__ __device__ static constexpr int opp(int q) { return MM::opp(q); }
};

struct AdjArgs {
    float *lam;  // adjoint state [50][N], FP32, AA layout of MMRev
    const float *eps, *mu, *sig;
    const float *E;  // forward E(f_n) [3][N]
    uint32_t nx, ny, nz, N;
    int32_t det_z;
    double *g_eps, *g_sig;  // [N] accumulators
    const float *E0, *B0;   // initial fields (only on the last adjoint step), or null
};

// One adjoint step for one cell: mu (pre-collision adjoint, overwritten with
// lambda), the forward field E of the same time level, the media; returns the
// gradient contributions of this step.
__device__ __forceinline__ void mm_adjoint_cell(float (&mu)[50], const float E[3], const CellMedia &m, bool plane,
                                                const float *E0c, float &gE, float &gS) {
    const float a = m.eps_r + 0.5f * m.sigma;
    const float ia = 1.0f / a;
    // adjoint moments of the moving populations
    float Mv[3] = {0.f, 0.f, 0.f}, Me0[3] = {0.f, 0.f, 0.f}, Me1[3] = {0.f, 0.f, 0.f};
    float Mb0[3] = {0.f, 0.f, 0.f}, Mb1[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float u00 = mu[p * 8 + i * 2], u01 = mu[p * 8 + i * 2 + 1];
            const float u10 = mu[24 + p * 8 + i * 2], u11 = mu[24 + p * 8 + i * 2 + 1];
            const float s = (u00 + u01) + (u10 + u11);  // v_q is the same for j = 0, 1 and r = 0, 1
            const float d0 = u00 - u01, d1 = u10 - u11;  // e_{i1} = -e_{i0}, b_{i1} = -b_{i0}
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (kMMV[p][i][c] != 0) Mv[c] += kMMV[p][i][c] > 0 ? s : -s;
                if (mm_e2(p, i, c) != 0) {
                    Me0[c] += (mm_e2(p, i, c) > 0 ? 0.5f : -0.5f) * d0;
                    Me1[c] += (mm_e2(p, i, c) > 0 ? 0.5f : -0.5f) * d1;
                }
                if (kMMB[p][c] != 0) {
                    Mb0[c] += kMMB[p][c] > 0 ? d0 : -d0;
                    Mb1[c] += kMMB[p][c] > 0 ? d1 : -d1;
                }
            }
        }
    // gradient of C through f_eq: d f_eq^(0) = v.dJ/16 + d(eps_r E).e/4, d f_eq^(1) = v.dJ/16 + dE.e/4
    // with E = D'/a, J = sigma E, a = eps_r + sigma/2
    float vMvE = 0.f, vMe0E = 0.f, vMe1E = 0.f, E2 = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        vMvE += Mv[c] * E[c];
        vMe0E += Me0[c] * E[c];
        vMe1E += Me1[c] * E[c];
        E2 += E[c] * E[c];
    }
    // d/d eps_r: dE = -E/a, dJ = -sigma E/a, d(eps_r E) = E sigma/(2a)
    gE = 2.f * ia * (-m.sigma * vMvE * 0.0625f + 0.5f * m.sigma * vMe0E * 0.25f - vMe1E * 0.25f);
    // d/d sigma: dE = -E/(2a), dJ = eps_r E / a, d(eps_r E) = -eps_r E/(2a)
    gS = 2.f * ia * (m.eps_r * vMvE * 0.0625f - 0.5f * m.eps_r * vMe0E * 0.25f - 0.5f * vMe1E * 0.25f);
    if (plane) {
        // l = |E|^2: dl/deps_r = -2|E|^2/a, dl/dsigma = -|E|^2/a
        gE -= 2.f * E2 * ia;
        gS -= E2 * ia;
    }
    // C^T mu = 2 M^T (U^T mu) - mu
    float GD[3], GB[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        GD[c] = ia * (m.sigma * 0.0625f * Mv[c] + 0.25f * m.eps_r * Me0[c] + 0.25f * Me1[c]);
        GB[c] = Mb0[c] * (0.125f / m.mu_r) + 0.125f * Mb1[c];
    }
    const float Grho = mu[48] + mu[49];
    // dl/df for r = 0 moving populations: 2 E . e_q / a (through D')
    float LD[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) LD[c] = plane ? 2.f * E[c] * ia : 0.f;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float gb = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (kMMB[p][c] != 0) gb += kMMB[p][c] > 0 ? GB[c] : -GB[c];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float ge = 0.f, le = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (mm_e2(p, i, c) != 0) {
                    ge += mm_e2(p, i, c) > 0 ? GD[c] : -GD[c];
                    le += mm_e2(p, i, c) > 0 ? LD[c] : -LD[c];
                }
            ge *= 0.5f;  // GD . e_{i0}
            le *= 0.5f;  // LD . e_{i0}
            const int q0 = p * 8 + i * 2, q1 = 24 + p * 8 + i * 2;
            mu[q0] = 2.f * (ge + Grho) - mu[q0] + le;
            mu[q0 + 1] = 2.f * (-ge + Grho) - mu[q0 + 1] - le;
            mu[q1] = 2.f * gb - mu[q1];
            mu[q1 + 1] = -2.f * gb - mu[q1 + 1];
        }
    }
    mu[48] = 2.f * Grho - mu[48];
    mu[49] = -mu[49];
    if (E0c) {
        // f_0 = f_eq(E0, B0): d f_0^(0)_q / d eps_r = E0 . e_q / 4
        float Le0[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float d0 = mu[p * 8 + i * 2] - mu[p * 8 + i * 2 + 1];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (mm_e2(p, i, c) != 0) Le0[c] += (mm_e2(p, i, c) > 0 ? 0.5f : -0.5f) * d0;
            }
        gE += 0.25f * (E0c[0] * Le0[0] + E0c[1] * Le0[1] + E0c[2] * Le0[2]);
    }
}

template <int ODD>
__global__ __launch_bounds__(kBlock) void mm_adjoint_kernel(AdjArgs a) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.N) return;
    const uint32_t nxy = a.nx * a.ny;
    const uint32_t z = c / nxy, rem = c - z * nxy, y = rem / a.nx, x = rem - y * a.nx;
    const Nbr nb = make_nbr(c, x, y, z, a.nx, a.ny, a.nz);
    const size_t N = a.N;
    float mu[50];
    gather<MMRev, ODD, StF32>(a.lam, N, nb, mu, 1.f);
    const float E[3] = {a.E[c], a.E[N + c], a.E[2 * N + c]};
    const CellMedia m{a.eps[c], a.mu[c], a.sig[c]};
    float E0c[3];
    if (a.E0) {
        E0c[0] = a.E0[c];
        E0c[1] = a.E0[N + c];
        E0c[2] = a.E0[2 * N + c];
    }
    float gE, gS;
    mm_adjoint_cell(mu, E, m, int32_t(z) == a.det_z, a.E0 ? E0c : nullptr, gE, gS);
    a.g_eps[c] += double(gE);
    a.g_sig[c] += double(gS);
    scatter<MMRev, ODD, StF32>(a.lam, N, nb, mu, 1.f);
}

__global__ void scale_grads(double *g, double s, size_t n) {
    const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) g[i] *= s;
}

struct AdjLayout {
    size_t ckpt, frames, lam, total, state_bytes;
    int64_t S;
};

AdjLayout adj_layout(const lbem_desc *d, int64_t nsteps, int32_t K) {
    AdjLayout L{};
    const size_t N = size_t(d->nx) * d->ny * d->nz;
    L.state_bytes = N * (d->model == LBEM_MM ? 50 : 36) * (d->storage == LBEM_F32 ? 4 : 2);
    L.S = (nsteps + K - 1) / K;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    L.ckpt = off;
    off = al(off + size_t(L.S + 1) * al(L.state_bytes));
    L.frames = off;
    off = al(off + size_t(K) * 3 * N * 4);
    L.lam = off;
    off = al(off + N * 50 * 4);
    L.total = off;
    return L;
}

uint32_t grid256(size_t n) { return uint32_t((n + kBlock - 1) / kBlock); }

}  // namespace

lbem_status lbem_adjoint_workspace_size(const lbem_desc *desc, int64_t nsteps, int32_t K, size_t *bytes) {
    size_t dummy;
    lbem_status st = lbem_workspace_size(desc, &dummy);
    if (st) return st;
    if (!bytes) return fail(LBEM_EINVAL, "bytes is NULL");
    if (nsteps < 1 || K < 1) return fail(LBEM_EINVAL, "nsteps and K must be >= 1");
    *bytes = adj_layout(desc, nsteps, K).total;
    return LBEM_OK;
}

lbem_status lbem_adjoint_forward(lbem_lattice *lat, int64_t nsteps, int32_t K, int32_t det_z, void *ws,
                                 size_t ws_bytes, double *loss) {
    if (!lat || !ws || !loss) return fail(LBEM_EINVAL, "null argument");
    if (nsteps < 1 || K < 1) return fail(LBEM_EINVAL, "nsteps and K must be >= 1");
    if (lat->d.model != LBEM_MM) return fail(LBEM_ESTATE, "the adjoint is provided for the MM model");
    if (lat->nsrc > 0 || lat->plane_z >= 0) return fail(LBEM_ESTATE, "the adjoint needs a lattice without sources");
    if (det_z < 0 || det_z >= lat->d.nz) return fail(LBEM_EINVAL, "detector plane z = %d outside the lattice", det_z);
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(LBEM_EINVAL, "workspace must be 256-byte aligned");
    const AdjLayout L = adj_layout(&lat->d, nsteps, K);
    if (ws_bytes < L.total) return fail(LBEM_ENOMEM, "adjoint workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    char *w = static_cast<char *>(ws);
    lbem_status st = lbem_set_detector(lat, det_z);
    if (st) return st;
    lat->adj_ws = nullptr;
    const int64_t t0 = lat->t;
    const size_t sb = (L.state_bytes + 255) & ~size_t(255);
    for (int64_t s = 0; s < L.S; ++s) {
        st = lbem_save_state(lat, w + L.ckpt + size_t(s) * sb);
        if (!st) st = lbem_step(lat, std::min<int64_t>(K, nsteps - s * K));
        if (st) return st;
    }
    st = lbem_save_state(lat, w + L.ckpt + size_t(L.S) * sb);
    if (!st) st = lbem_detector_read(lat, loss);
    if (st) return st;
    lat->adj_ws = ws;
    lat->adj_t0 = t0;
    lat->adj_nsteps = nsteps;
    lat->adj_K = K;
    lat->adj_det = det_z;
    return LBEM_OK;
}

lbem_status lbem_adjoint_backward(lbem_lattice *lat, void *ws, size_t ws_bytes, const float *E0, const float *B0,
                                  double scale, double *grad_eps, double *grad_sigma) {
    if (!lat || !ws || !grad_eps || !grad_sigma) return fail(LBEM_EINVAL, "null argument");
    if (lat->adj_ws != ws) return fail(LBEM_ESTATE, "no lbem_adjoint_forward recorded in this workspace");
    if ((E0 == nullptr) != (B0 == nullptr)) return fail(LBEM_EINVAL, "give both E0 and B0 or neither");
    const int64_t nsteps = lat->adj_nsteps, t0 = lat->adj_t0;
    const int32_t K = lat->adj_K;
    const AdjLayout L = adj_layout(&lat->d, nsteps, K);
    if (ws_bytes < L.total) return fail(LBEM_ENOMEM, "adjoint workspace too small");
    char *w = static_cast<char *>(ws);
    const size_t sb = (L.state_bytes + 255) & ~size_t(255);
    const size_t N = lat->N;
    hipStream_t s = lat->stream;
    // gradients and the adjoint state start at zero
    hipLaunchKernelGGL(zero_bytes, dim3(grid256(2 * N)), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(grad_eps), 2 * N);
    hipLaunchKernelGGL(zero_bytes, dim3(grid256(2 * N)), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(grad_sigma), 2 * N);
    hipLaunchKernelGGL(zero_bytes, dim3(grid256(50 * N)), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(w + L.lam), 50 * N);
    lbem_status st = hip_check(hipGetLastError(), "zero");
    if (st) return st;
    float *frames = reinterpret_cast<float *>(w + L.frames);
    AdjArgs aa{};
    aa.lam = reinterpret_cast<float *>(w + L.lam);
    aa.eps = reinterpret_cast<const float *>(lat->ws + lat->L.eps);
    aa.mu = reinterpret_cast<const float *>(lat->ws + lat->L.mu);
    aa.sig = reinterpret_cast<const float *>(lat->ws + lat->L.sig);
    aa.nx = lat->d.nx;
    aa.ny = lat->d.ny;
    aa.nz = lat->d.nz;
    aa.N = lat->N;
    aa.det_z = lat->adj_det;
    aa.g_eps = grad_eps;
    aa.g_sig = grad_sigma;
    int64_t j = 0;  // adjoint steps done (parity of the adjoint AA layout)
    for (int64_t seg = L.S - 1; seg >= 0; --seg) {
        const int64_t tseg = t0 + seg * K;
        const int64_t ks = std::min<int64_t>(K, nsteps - seg * K);
        st = lbem_load_state(lat, w + L.ckpt + size_t(seg) * sb, tseg);
        if (st) return st;
        // recompute the segment, keeping E(f_n) of every step
        StepArgs a = base_step_args(lat);
        for (int64_t k = 0; k < ks; ++k) {
            a.E_out = frames + size_t(k) * 3 * N;
            dispatch_step(lat, a, int(lat->t & 1));
            st = hip_check(hipGetLastError(), "recompute launch");
            if (st) return st;
            lat->t += 1;
        }
        // adjoint steps of the segment, last time level first
        for (int64_t k = ks - 1; k >= 0; --k) {
            aa.E = frames + size_t(k) * 3 * N;
            const bool first = seg == 0 && k == 0;
            aa.E0 = first ? E0 : nullptr;
            aa.B0 = first ? B0 : nullptr;
            if (j & 1) hipLaunchKernelGGL(mm_adjoint_kernel<1>, dim3(grid256(N)), dim3(kBlock), 0, s, aa);
            else hipLaunchKernelGGL(mm_adjoint_kernel<0>, dim3(grid256(N)), dim3(kBlock), 0, s, aa);
            st = hip_check(hipGetLastError(), "adjoint launch");
            if (st) return st;
            ++j;
        }
    }
    if (scale != 1.0) {
        hipLaunchKernelGGL(scale_grads, dim3(grid256(N)), dim3(kBlock), 0, s, grad_eps, scale, N);
        hipLaunchKernelGGL(scale_grads, dim3(grid256(N)), dim3(kBlock), 0, s, grad_sigma, scale, N);
    }
    // leave the lattice as the forward left it
    st = lbem_load_state(lat, w + L.ckpt + size_t(L.S) * sb, t0 + nsteps);
    if (st) return st;
    return hip_check(hipGetLastError(), "adjoint");
}
