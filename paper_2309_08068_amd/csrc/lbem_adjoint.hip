// lbem_adjoint.hip -- reverse-time (adjoint) differentiation of the
// detector-plane loss with respect to the per-cell eps_r and sigma, for the MM
// and the modified HV model.
//
// Forward, for fixed media theta = (eps_r, sigma):  f_{n+1} = S C_theta f_n,
// with C(f) = 2 f_eq(m(f); theta) - f (+ T for HV; Sections II-III) and S the
// advection.
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
#include <mutex>

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

// MM in difference form with every velocity reversed.
struct MMDRev {
    static constexpr int Q = 24;
    __host__ __device__ static constexpr int vel(int q, int a) { return -MMD::vel(q, a); }
    __host__ __device__ static constexpr int opp(int q) { return MMD::opp(q); }
};

// HV with every velocity reversed.
struct HVRev {
    static constexpr int Q = 36;
    __host__ __device__ static constexpr int vel(int q, int a) { return -HV::vel(q, a); }
    __host__ __device__ static constexpr int opp(int q) { return HV::opp(q); }
};

struct AdjArgs {
    float *lam;  // adjoint state, FP32, the populations' layout, AA order of the reversed velocities
    PopLayout pl;
    const float *eps, *mu, *sig;
    const float *E;  // forward E(f_n) [3][N]
    uint32_t nx, ny, nz, N;
    int32_t det_z;
    float *g_eps, *g_sig;  // [N] FP32 accumulators of the current segment
    const float *E0, *B0;  // initial fields (only on the last adjoint step), or null
};

// One adjoint step for one cell: mu (pre-collision adjoint, overwritten with
// lambda), the forward field E of the same time level, the media; returns the
// gradient contributions of this step.
__device__ __forceinline__ void mm_adjoint_cell(float (&mu)[50], const float E[3], const CellMedia &m, bool plane,
                                                bool first, const float (&E0c)[3], float &gE, float &gS) {
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
    if (first) {
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


// One HV adjoint step for one cell.  With D = sum e_i, B = sum h_i, E = D/eps,
// H = B/mu, J = sigma E (eqs. MacroscopicFieldsHV, equilibriumHV,
// CollisionmodifiedHV):  e'_i = D/3 - v_i x H - e_i - (J.v_i) v_i / 2,
// h'_i = B/3 + v_i x E - h_i.  With S_e = sum mu_e_i, S_h = sum mu_h_i,
// A = sum (mu_e_i . v_i) v_i, W = sum mu_h_i x v_i, Y = sum mu_e_i x v_i:
//   (C^T mu)_e_j = S_e/3 - (sigma/eps) A/2 + W/eps - mu_e_j,
//   (C^T mu)_h_j = S_h/3 - Y/mu - mu_h_j,
// and the collision's dependence on theta through E and J gives
//   dL/deps_r += (sigma/(2 eps_r)) E.A - E.W / eps_r,   dL/dsigma += -E.A/2.
__device__ __forceinline__ void hv_adjoint_cell(float (&mu)[36], const float E[3], const CellMedia &m, bool plane,
                                                bool first, const float (&E0c)[3], float &gE, float &gS) {
    const float eps = kHVEps0 * m.eps_r, mmu = kHVMu0 * m.mu_r;
    float Se[3] = {0.f, 0.f, 0.f}, Sh[3] = {0.f, 0.f, 0.f}, A[3] = {0.f, 0.f, 0.f};
    float W[3] = {0.f, 0.f, 0.f}, Y[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const float ue[3] = {mu[3 * i], mu[3 * i + 1], mu[3 * i + 2]};
        const float uh[3] = {mu[18 + 3 * i], mu[18 + 3 * i + 1], mu[18 + 3 * i + 2]};
        const int v[3] = {kHVV[i][0], kHVV[i][1], kHVV[i][2]};
        float uv = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Se[c] += ue[c];
            Sh[c] += uh[c];
            if (v[c] != 0) uv += v[c] > 0 ? ue[c] : -ue[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (v[c] != 0) A[c] += v[c] > 0 ? uv : -uv;
            // (u x v)_c = u_{c+1} v_{c+2} - u_{c+2} v_{c+1}
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            W[c] += uh[c1] * float(v[c2]) - uh[c2] * float(v[c1]);
            Y[c] += ue[c1] * float(v[c2]) - ue[c2] * float(v[c1]);
        }
    }
    const float EA = E[0] * A[0] + E[1] * A[1] + E[2] * A[2];
    const float EW = E[0] * W[0] + E[1] * W[1] + E[2] * W[2];
    const float E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
    gE = (0.5f * m.sigma * EA - EW) / m.eps_r;
    gS = -0.5f * EA;
    if (plane) gE -= 2.f * E2 / m.eps_r;  // l = |E|^2, E = D / (eps0 eps_r)
    float Ge[3], Gh[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Ge[c] = Se[c] * (1.f / 3.f) - 0.5f * (m.sigma / eps) * A[c] + W[c] / eps + (plane ? 2.f * E[c] / eps : 0.f);
        Gh[c] = Sh[c] * (1.f / 3.f) - Y[c] / mmu;
    }
    float Le[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            mu[3 * i + c] = Ge[c] - mu[3 * i + c];
            mu[18 + 3 * i + c] = Gh[c] - mu[18 + 3 * i + c];
            Le[c] += mu[3 * i + c];
        }
    if (first) {
        // e_i(0) = (eps E0 - 3 v_i x H0) / 6:  d e_i(0) / d eps_r = E0 / 2
        gE += 0.5f * (E0c[0] * Le[0] + E0c[1] * Le[1] + E0c[2] * Le[2]);
    }
}

template <class M>
struct AdjCell;
template <>
struct AdjCell<MM> {
    using Rev = MMRev;
    __device__ static void step(float (&mu)[50], const float E[3], const CellMedia &m, bool plane, bool first,
                                const float (&E0c)[3], float &gE, float &gS) {
        mm_adjoint_cell(mu, E, m, plane, first, E0c, gE, gS);
    }
};
// MM in difference form: the collision d' = 4 u(E(d), B(d)) - d is linear in
// d; with adjoint moments Me_r = sum_i e_{i0} mu^(r)_i and Mb_r = sum_i b_{i0}
// mu^(r)_i (E = D'/a, a = eps_r + sigma/2) its transpose is
//   lambda^(0)_i = e_{i0} . (eps_r Me_0 + Me_1) / a - mu^(0)_i,
//   lambda^(1)_i = b_{i0} . (Mb_0 / (2 mu_r) + Mb_1 / 2) - mu^(1)_i,
// and mu . d' depends on theta through E only.  The sums f_{i0} + f_{i1} of
// the full scheme never reach E, so their adjoint is zero and this is the MM
// adjoint restricted to the differences.
__device__ __forceinline__ void mmd_adjoint_cell(float (&mu)[24], const float E[3], const CellMedia &m, bool plane,
                                                 bool first, const float (&E0c)[3], float &gE, float &gS) {
    const float a = m.eps_r + 0.5f * m.sigma;
    const float ia = 1.0f / a;
    float Me0[3] = {0.f, 0.f, 0.f}, Me1[3] = {0.f, 0.f, 0.f}, Mb0[3] = {0.f, 0.f, 0.f}, Mb1[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float d0 = mu[p * 4 + i], d1 = mu[12 + p * 4 + i];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
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
    float Me0E = 0.f, Me1E = 0.f, E2 = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Me0E += Me0[c] * E[c];
        Me1E += Me1[c] * E[c];
        E2 += E[c] * E[c];
    }
    // d/d eps_r: dE = -E/a; d/d sigma: dE = -E/(2a)
    gE = ia * (0.5f * m.sigma * Me0E - Me1E);
    gS = -0.5f * ia * (m.eps_r * Me0E + Me1E);
    if (plane) {
        gE -= 2.f * E2 * ia;
        gS -= E2 * ia;
    }
    float GD[3], GB[3], LD[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        GD[c] = ia * (m.eps_r * Me0[c] + Me1[c]);
        GB[c] = Mb0[c] * (0.5f / m.mu_r) + 0.5f * Mb1[c];
        LD[c] = plane ? 2.f * E[c] * ia : 0.f;  // dl/dD' = 2 E / a
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float gb = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (kMMB[p][c] != 0) gb += kMMB[p][c] > 0 ? GB[c] : -GB[c];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float ge = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (mm_e2(p, i, c) != 0) ge += mm_e2(p, i, c) > 0 ? GD[c] + LD[c] : -(GD[c] + LD[c]);
            mu[p * 4 + i] = 0.5f * ge - mu[p * 4 + i];
            mu[12 + p * 4 + i] = gb - mu[12 + p * 4 + i];
        }
    }
    if (first) {
        // d_0 = 2 u(E0, B0): d d^(0)_i / d eps_r = E0 . e_{i0} / 2
        float Le0[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (mm_e2(p, i, c) != 0) Le0[c] += (mm_e2(p, i, c) > 0 ? 0.5f : -0.5f) * mu[p * 4 + i];
        gE += 0.5f * (E0c[0] * Le0[0] + E0c[1] * Le0[1] + E0c[2] * Le0[2]);
    }
}

template <>
struct AdjCell<MMD> {
    using Rev = MMDRev;
    __device__ static void step(float (&mu)[24], const float E[3], const CellMedia &m, bool plane, bool first,
                                const float (&E0c)[3], float &gE, float &gS) {
        mmd_adjoint_cell(mu, E, m, plane, first, E0c, gE, gS);
    }
};

template <>
struct AdjCell<HV> {
    using Rev = HVRev;
    __device__ static void step(float (&mu)[36], const float E[3], const CellMedia &m, bool plane, bool first,
                                const float (&E0c)[3], float &gE, float &gS) {
        hv_adjoint_cell(mu, E, m, plane, first, E0c, gE, gS);
    }
};

template <class M, int ODD>
__global__ __launch_bounds__(kBlock) void adjoint_kernel(AdjArgs a) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.N) return;
    const uint32_t nxy = a.nx * a.ny;
    const uint32_t z = c / nxy, rem = c - z * nxy, y = rem / a.nx, x = rem - y * a.nx;
    const Nbr nb = make_nbr(c, x, y, z, a.nx, a.ny, a.nz);
    const size_t N = a.N;
    const size_t P = a.pl.C;  // plane stride (generic lattices are a single chunk)
    using R = typename AdjCell<M>::Rev;
    float mu[M::Q];
    gather<R, ODD, StF32>(a.lam, P, nb, mu, 1.f);
    const float E[3] = {__builtin_nontemporal_load(a.E + c), __builtin_nontemporal_load(a.E + N + c),
                        __builtin_nontemporal_load(a.E + 2 * N + c)};
    const CellMedia m{a.eps[c], a.mu[c], a.sig[c]};
    float E0c[3] = {0.f, 0.f, 0.f};
    if (a.E0) {
        E0c[0] = a.E0[c];
        E0c[1] = a.E0[N + c];
        E0c[2] = a.E0[2 * N + c];
    }
    float gE, gS;
    AdjCell<M>::step(mu, E, m, int32_t(z) == a.det_z, a.E0 != nullptr, E0c, gE, gS);
    a.g_eps[c] += gE;
    a.g_sig[c] += gS;
    Nbr nb2 = nb;
    float *lam2 = a.lam;
    late_addresses(nb2, lam2, mu[0]);
    scatter<R, ODD, StF32>(lam2, P, nb2, mu, 1.f);
}

// Row form of the adjoint step (one block per x-row, see RowIO); LATE and
// DIRECT as for the forward row kernel.
template <class M, int ODD, int RB, int LATE, int DIRECT>
__global__ __launch_bounds__(RB) void adjoint_row_kernel(AdjArgs a) {
    using R = typename AdjCell<M>::Rev;
    __shared__ float sh[(ODD && !DIRECT) ? n_xshift<R>() : 1][RB];
    const uint32_t row = blockIdx.x;
    const uint32_t z = row / a.ny;
    const bool live = threadIdx.x < a.nx;  // rows shorter than RB leave the last threads idle
    const uint32_t c = row * a.nx + (live ? threadIdx.x : 0u);
    const size_t N = a.N;
    RowIO<R, StF32, RB> io(a.lam, a.pl, a.ny, a.nz, row);
    float mu[M::Q];
    if (DIRECT) io.template gather_direct<ODD>(mu, 1.f);
    else io.template gather<ODD>(mu, sh, 1.f);
    const float E[3] = {__builtin_nontemporal_load(a.E + c), __builtin_nontemporal_load(a.E + N + c),
                        __builtin_nontemporal_load(a.E + 2 * N + c)};
    const CellMedia m{a.eps[c], a.mu[c], a.sig[c]};
    float E0c[3] = {0.f, 0.f, 0.f};
    if (a.E0) {
        E0c[0] = a.E0[c];
        E0c[1] = a.E0[N + c];
        E0c[2] = a.E0[2 * N + c];
    }
    float gE, gS;
    AdjCell<M>::step(mu, E, m, int32_t(z) == a.det_z, a.E0 != nullptr, E0c, gE, gS);
    if (live) {
        a.g_eps[c] += gE;
        a.g_sig[c] += gS;
    }
    if (LATE) io.late(mu[0]);
    if (DIRECT) io.template scatter_direct<ODD>(mu, 1.f);
    else io.template scatter<ODD>(mu, sh, 1.f);
}

// g64 += scale * g32 and g32 = 0 (end of a segment; FP64 across segments)
__global__ void flush_grads(double *g64e, double *g64s, float *g32e, float *g32s, double scale, size_t n) {
    const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    g64e[i] += scale * double(g32e[i]);
    g64s[i] += scale * double(g32s[i]);
    g32e[i] = 0.f;
    g32s[i] = 0.f;
}

struct AdjLayout {
    size_t ckpt, frames, lam, g32, total, state_bytes;
    int64_t S, keep;  // segments, and trailing segments whose frames the forward keeps
};

AdjLayout adj_layout(const lbem_desc *d, int64_t nsteps, int32_t K, int32_t keep) {
    AdjLayout L{};
    const size_t N = size_t(d->nx) * d->ny * d->nz;
    L.state_bytes = state_bytes(d);
    L.S = (nsteps + K - 1) / K;
    L.keep = std::max<int64_t>(1, std::min<int64_t>(keep, L.S));
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    L.ckpt = off;
    off = al(off + size_t(L.S + 1) * al(L.state_bytes));
    L.frames = off;
    off = al(off + size_t(L.keep) * size_t(K) * 3 * N * 4);
    L.lam = off;
    off = al(off + size_t(pop_elems(d)) * 4);
    L.g32 = off;
    off = al(off + N * 2 * 4);
    L.total = off;
    return L;
}

uint32_t grid256(size_t n) { return uint32_t((n + kBlock - 1) / kBlock); }

template <class M, int ODD, int RB>
const void *adjoint_row_ptr(int form) {
    switch (form) {
        case 0: return reinterpret_cast<const void *>(&adjoint_row_kernel<M, ODD, RB, 0, 0>);
        case 1: return reinterpret_cast<const void *>(&adjoint_row_kernel<M, ODD, RB, 1, 0>);
        default: return reinterpret_cast<const void *>(&adjoint_row_kernel<M, ODD, RB, 1, 1>);
    }
}

template <class M, int ODD>
const void *adjoint_ptr_p(uint32_t rb, int form) {
    switch (rb) {
        case 128: return adjoint_row_ptr<M, ODD, 128>(form);
        case 256: return adjoint_row_ptr<M, ODD, 256>(form);
        case 384: return adjoint_row_ptr<M, ODD, 384>(form);
        case 512: return adjoint_row_ptr<M, ODD, 512>(form);
        default: return reinterpret_cast<const void *>(&adjoint_kernel<M, ODD>);
    }
}

const void *adjoint_ptr(const lbem_lattice *lat, int odd, int form) {
    const uint32_t rb = row_block(&lat->d);
    if (lat->d.model == LBEM_MM) return odd ? adjoint_ptr_p<MM, 1>(rb, form) : adjoint_ptr_p<MM, 0>(rb, form);
    if (lat->d.model == LBEM_MM_DIFF) return odd ? adjoint_ptr_p<MMD, 1>(rb, form) : adjoint_ptr_p<MMD, 0>(rb, form);
    return odd ? adjoint_ptr_p<HV, 1>(rb, form) : adjoint_ptr_p<HV, 0>(rb, form);
}

void launch_adjoint(const lbem_lattice *lat, const AdjArgs &aa, int odd, int form, size_t pad) {
    const uint32_t rb = row_block(&lat->d);
    void *args[] = {const_cast<AdjArgs *>(&aa)};
    (void)hipLaunchKernel(adjoint_ptr(lat, odd, form), dim3(rb ? lat->nblocks : grid256(lat->N)),
                          dim3(rb ? rb : kBlock), args, pad, lat->stream);
}

// Choose the adjoint row kernel's form and occupancy cap per parity by timing
// a few launches on the workspace (whose adjoint state and accumulators the
// caller clears afterwards).
lbem_status tune_adjoint(lbem_lattice *lat, const AdjArgs &aa) {
    lat->adj_tuned = 1;
    for (int p = 0; p < 2; ++p) {
        lat->adj_form[p] = 1;
        lat->adj_cap[p] = 0;
        lat->adj_pad[p] = 0;
    }
    if (!row_block(&lat->d)) return LBEM_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lbem_status st = hip_check(hipEventCreate(&e0), "event");
    if (!st) st = hip_check(hipEventCreate(&e1), "event");
    static const int caps[] = {0, 2, 3, 4};
    for (int p = 0; p < 2 && !st; ++p) {
        float best = 1e30f;
        for (int form = 0; form < 3 && !st; ++form)
            for (int cap : caps) {
                const size_t pad = lds_pad_for(adjoint_ptr(lat, p, form), cap);
                launch_adjoint(lat, aa, p, form, pad);  // warm-up
                st = hip_check(hipEventRecord(e0, lat->stream), "record");
                for (int k = 0; k < 3 && !st; ++k) launch_adjoint(lat, aa, p, form, pad);
                if (!st) st = hip_check(hipGetLastError(), "trial launch");
                if (!st) st = hip_check(hipEventRecord(e1, lat->stream), "record");
                if (!st) st = hip_check(hipEventSynchronize(e1), "sync");
                float ms = 0.f;
                if (!st) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
                if (!st && ms < best) {
                    best = ms;
                    lat->adj_form[p] = form;
                    lat->adj_cap[p] = cap;
                    lat->adj_pad[p] = pad;
                }
            }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

lbem_status lbem_adjoint_workspace_size(const lbem_desc *desc, int64_t nsteps, int32_t K, int32_t keep,
                                        size_t *bytes) {
    size_t dummy;
    lbem_status st = lbem_workspace_size(desc, &dummy);
    if (st) return st;
    if (!bytes) return fail(LBEM_EINVAL, "bytes is NULL");
    if (nsteps < 1 || K < 1 || keep < 1) return fail(LBEM_EINVAL, "nsteps, K and keep must be >= 1");
    if (desc->storage != LBEM_F32) return fail(LBEM_EINVAL, "the adjoint needs FP32 population storage");
    *bytes = adj_layout(desc, nsteps, K, keep).total;
    return LBEM_OK;
}

lbem_status lbem_adjoint_keep(const lbem_desc *desc, int64_t nsteps, int32_t K, size_t budget_bytes,
                              int32_t *keep) {
    size_t dummy;
    lbem_status st = lbem_adjoint_workspace_size(desc, nsteps, K, 1, &dummy);
    if (st) return st;
    if (!keep) return fail(LBEM_EINVAL, "keep is NULL");
    if (dummy > budget_bytes) return fail(LBEM_ENOMEM, "even keep = 1 needs %zu bytes", dummy);
    // the workspace grows with keep: the largest keep that fits, by bisection
    int64_t lo = 1, hi = std::min<int64_t>((nsteps + K - 1) / K, INT32_MAX);
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (adj_layout(desc, nsteps, K, int32_t(mid)).total <= budget_bytes) lo = mid;
        else hi = mid - 1;
    }
    *keep = int32_t(lo);
    return LBEM_OK;
}

lbem_status lbem_adjoint_forward(lbem_lattice *lat, int64_t nsteps, int32_t K, int32_t keep, int32_t det_z, void *ws,
                                 size_t ws_bytes, double *loss) {
    if (!lat || !ws || !loss) return fail(LBEM_EINVAL, "null argument");
    if (nsteps < 1 || K < 1 || keep < 1) return fail(LBEM_EINVAL, "nsteps, K and keep must be >= 1");
    // the reverse kernels differentiate the unrounded FP32 step, which is the
    // forward map only when nothing is rounded to 16 bits between steps
    if (lat->d.storage != LBEM_F32) return fail(LBEM_EINVAL, "the adjoint needs FP32 population storage");
    if (lat->nsrc > 0 || lat->plane_z >= 0) return fail(LBEM_ESTATE, "the adjoint needs a lattice without sources");
    if (det_z < 0 || det_z >= lat->d.nz) return fail(LBEM_EINVAL, "detector plane z = %d outside the lattice", det_z);
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(LBEM_EINVAL, "workspace must be 256-byte aligned");
    const AdjLayout L = adj_layout(&lat->d, nsteps, K, keep);
    if (ws_bytes < L.total) return fail(LBEM_ENOMEM, "adjoint workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    char *w = static_cast<char *>(ws);
    lbem_status st = lbem_set_detector(lat, det_z);
    if (st) return st;
    lat->adj_ws = nullptr;
    const int64_t t0 = lat->t;
    const size_t sb = (L.state_bytes + 255) & ~size_t(255);
    float *frames = reinterpret_cast<float *>(w + L.frames);
    for (int64_t s = 0; s < L.S; ++s) {
        const int64_t ks = std::min<int64_t>(K, nsteps - s * K);
        st = lbem_save_state(lat, w + L.ckpt + size_t(s) * sb);
        if (st) return st;
        // the last `keep` segments also keep E(f_n) of each step, so the
        // reverse pass does not recompute them
        const int64_t slot = s - (L.S - L.keep);
        st = step_impl(lat, ks, slot >= 0 ? frames + size_t(slot) * K * 3 * lat->N : nullptr);
        if (st) return st;
    }
    st = lbem_save_state(lat, w + L.ckpt + size_t(L.S) * sb);
    if (!st) st = lbem_detector_read(lat, loss);
    if (st) return st;
    lat->adj_ws = ws;
    lat->adj_t0 = t0;
    lat->adj_nsteps = nsteps;
    lat->adj_K = K;
    lat->adj_keep = int32_t(L.keep);
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
    const AdjLayout L = adj_layout(&lat->d, nsteps, K, lat->adj_keep);
    if (ws_bytes < L.total) return fail(LBEM_ENOMEM, "adjoint workspace too small");
    char *w = static_cast<char *>(ws);
    const size_t sb = (L.state_bytes + 255) & ~size_t(255);
    const size_t N = lat->N;
    hipStream_t s = lat->stream;
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
    aa.pl = lat->pl;
    aa.det_z = lat->adj_det;
    aa.g_eps = reinterpret_cast<float *>(w + L.g32);
    aa.g_sig = aa.g_eps + N;
    if (!lat->adj_tuned) {
        aa.E = frames;  // any frame: the trial launches only need valid memory
        lbem_status st = tune_adjoint(lat, aa);
        if (st) return st;
    }
    // gradients and the adjoint state start at zero
    hipLaunchKernelGGL(zero_bytes, dim3(grid256(2 * N)), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(grad_eps), 2 * N);
    hipLaunchKernelGGL(zero_bytes, dim3(grid256(2 * N)), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(grad_sigma), 2 * N);
    const size_t lam_words = size_t(pop_elems(&lat->d));
    hipLaunchKernelGGL(zero_bytes, dim3(grid256(lam_words)), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(w + L.lam),
                       lam_words);
    hipLaunchKernelGGL(zero_bytes, dim3(grid256(2 * N)), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(w + L.g32), 2 * N);
    lbem_status st = hip_check(hipGetLastError(), "zero");
    if (st) return st;
    int64_t j = 0;  // adjoint steps done (parity of the adjoint AA layout)
    for (int64_t seg = L.S - 1; seg >= 0; --seg) {
        const int64_t tseg = t0 + seg * K;
        const int64_t ks = std::min<int64_t>(K, nsteps - seg * K);
        const int64_t slot = seg - (L.S - L.keep);
        float *segf = frames + size_t(slot >= 0 ? slot : 0) * K * 3 * N;
        if (slot < 0) {
            // recompute the segment, keeping E(f_n) of every step
            st = lbem_load_state(lat, w + L.ckpt + size_t(seg) * sb, tseg);
            if (st) return st;
            StepArgs a = base_step_args(lat);
            for (int64_t k = 0; k < ks; ++k) {
                a.E_out = segf + size_t(k) * 3 * N;
                dispatch_step(lat, a, int(lat->t & 1));
                st = hip_check(hipGetLastError(), "recompute launch");
                if (st) return st;
                lat->t += 1;
            }
        }
        // adjoint steps of the segment, last time level first
        for (int64_t k = ks - 1; k >= 0; --k) {
            aa.E = segf + size_t(k) * 3 * N;
            const bool first = seg == 0 && k == 0;
            aa.E0 = first ? E0 : nullptr;
            aa.B0 = first ? B0 : nullptr;
            const int odd = int(j & 1);
            launch_adjoint(lat, aa, odd, lat->adj_form[odd], lat->adj_pad[odd]);
            st = hip_check(hipGetLastError(), "adjoint launch");
            if (st) return st;
            ++j;
        }
        hipLaunchKernelGGL(flush_grads, dim3(grid256(N)), dim3(kBlock), 0, s, grad_eps, grad_sigma, aa.g_eps, aa.g_sig,
                           scale, N);
    }
    // leave the lattice as the forward left it
    st = lbem_load_state(lat, w + L.ckpt + size_t(L.S) * sb, t0 + nsteps);
    if (st) return st;
    return hip_check(hipGetLastError(), "adjoint");
}

lbem_status lbem_adjoint(lbem_lattice *lat, int64_t nsteps, int32_t K, int32_t keep, int32_t det_z, const float *E0,
                         const float *B0, double scale, double *grad_eps, double *grad_sigma, double *loss, void *ws,
                         size_t ws_bytes) {
    lbem_status st = lbem_adjoint_forward(lat, nsteps, K, keep, det_z, ws, ws_bytes, loss);
    if (st) return st;
    return lbem_adjoint_backward(lat, ws, ws_bytes, E0, B0, scale, grad_eps, grad_sigma);
}

lbem_status lbem_set_adjoint_tuning(lbem_lattice *lat, const int32_t *form, const int32_t *blocks_per_cu) {
    if (!lat || !form || !blocks_per_cu) return fail(LBEM_EINVAL, "null argument");
    for (int p = 0; p < 2; ++p) {
        if (form[p] < 0 || form[p] > 2) return fail(LBEM_EINVAL, "adjoint form must be 0, 1 or 2");
        if (blocks_per_cu[p] < 0 || blocks_per_cu[p] > 64) return fail(LBEM_EINVAL, "blocks_per_cu must be in [0, 64]");
    }
    for (int p = 0; p < 2; ++p) {
        lat->adj_form[p] = form[p];
        lat->adj_cap[p] = blocks_per_cu[p];
        lat->adj_pad[p] = lds_pad_for(adjoint_ptr(lat, p, form[p]), blocks_per_cu[p]);
    }
    lat->adj_tuned = 1;
    return LBEM_OK;
}

lbem_status lbem_get_adjoint_tuning(lbem_lattice *lat, int32_t *form, int32_t *blocks_per_cu) {
    if (!lat || !form || !blocks_per_cu) return fail(LBEM_EINVAL, "null argument");
    for (int p = 0; p < 2; ++p) {
        form[p] = lat->adj_tuned ? lat->adj_form[p] : -1;
        blocks_per_cu[p] = lat->adj_tuned ? lat->adj_cap[p] : -1;
    }
    return LBEM_OK;
}

// ------------------------------------------------------------------------
// lbem_adjoint_static: lbem_adjoint with its workspace in a fixed device
// array instead of a caller buffer, for callers that cannot allocate.
//
// `scratch` holds the checkpoints, frames, adjoint populations and FP32
// gradient accumulators that lbem_adjoint keeps in `ws`.  Each GPU has its own
// copy of the array; host code only ever uses the address that
// hipGetSymbolAddress returns for the current GPU (the array's name is a
// host-side stand-in, not a device address).  Nothing in it needs to start at
// zero: the forward writes every checkpoint and frame before the reverse pass
// reads it, and the reverse pass zeroes the adjoint populations and the
// accumulators itself.
// ------------------------------------------------------------------------
static constexpr size_t kStaticAdjointBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticAdjointBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Address of this GPU's scratch array (looked up once per device, with that
// device current).
lbem_status scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(LBEM_EINVAL, "device %d outside the supported range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        lbem_status st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st) return st;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LBEM_OK;
}
}  // namespace

size_t lbem_adjoint_static_bytes(void) { return kStaticAdjointBytes; }

lbem_status lbem_adjoint_static(lbem_lattice *lat, int64_t nsteps, int32_t K, int32_t keep, int32_t det_z,
                                const float *E0, const float *B0, double scale, double *grad_eps, double *grad_sigma,
                                double *loss) {
    if (!lat) return fail(LBEM_EINVAL, "lattice is NULL");
    if (nsteps < 1 || K < 1 || keep < 1) return fail(LBEM_EINVAL, "nsteps, K and keep must be >= 1");
    if (lat->d.storage != LBEM_F32) return fail(LBEM_EINVAL, "the adjoint needs FP32 population storage");
    const size_t need = adj_layout(&lat->d, nsteps, K, keep).total;
    if (need > kStaticAdjointBytes)
        return fail(LBEM_ENOMEM, "the adjoint of this lattice needs %zu bytes of workspace; the fixed one holds %zu",
                    need, kStaticAdjointBytes);
    int dev = -1;
    lbem_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev != lat->device)
        return fail(LBEM_EINVAL, "the lattice was created on GPU %d, GPU %d is current", lat->device, dev);
    void *ws = nullptr;
    st = scratch_address(dev, &ws);
    if (st) return st;
    // the first reverse pass of lbem_adjoint times launch variants with HIP
    // events; here a lattice without a tuning gets the row form with early
    // store addresses and no occupancy cap (every form gives the same bits)
    if (!lat->adj_tuned) {
        const int32_t form[2] = {0, 0}, cap[2] = {0, 0};
        st = lbem_set_adjoint_tuning(lat, form, cap);
        if (st) return st;
    }
    return lbem_adjoint(lat, nsteps, K, keep, det_z, E0, B0, scale, grad_eps, grad_sigma, loss, ws,
                        kStaticAdjointBytes);
}
