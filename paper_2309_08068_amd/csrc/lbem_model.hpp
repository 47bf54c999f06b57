// lbem_model.hpp -- lattice tables and the per-cell collision of the two
// Maxwell lattice-Boltzmann schemes, as device code for gfx950.
//
// Population numbering (shared by every kernel of this library):
//   MMD (MM in difference form): q = r * 12 + p * 4 + i for
//       d^{p(r)}_i = f^{p(r)}_{i0} - f^{p(r)}_{i1} (see MMD below).
//   MM: q = r * 24 + p * 8 + i * 2 + j for the moving populations f^{p(r)}_{ij}
//       (r = 0 electric, 1 magnetic; plane p = 0..2; direction i = 0..3 for the
//       paper's i = 1..4; j = 0, 1), q = 48 and 49 for the rest populations
//       f_0^(0), f_0^(1).
//   HV: q = r * 18 + i * 3 + a for component a of e_i (r = 0) or h_i (r = 1),
//       i = 0..5 for the paper's i = 1..6.
// The opposite of q (same r, j or component, reversed velocity) is the slot
// that the in-place AA streaming of the step kernels swaps with.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbem {

// ---------------------------------------------------------------- MM tables
// eq. (VelocitySetMiller): v_i^p = sqrt(2) (cos, sin)((2i - 1) pi / 4) in the
// plane p (xy, xz, yz).  The components are exactly 0 or +-1.
constexpr int kMMV[3][4][3] = {
    {{1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}},
    {{1, 0, 1}, {-1, 0, 1}, {-1, 0, -1}, {1, 0, -1}},
    {{0, 1, 1}, {0, -1, 1}, {0, -1, -1}, {0, 1, -1}},
};
// eq. (ElectromagneticVectorsMiller): e_{i0} = v_{[(i+2) mod 4]+1} / 2 in the
// paper's 1-based i, i.e. 2 e_{i0} = v[(i + 3) mod 4] for 0-based i, and
// e_{i1} = -e_{i0}.  b_{ij} = v_i x e_{ij} is the same for all i of a plane:
// b_{i0} = kMMB[p], b_{i1} = -kMMB[p].
constexpr int mm_e2(int p, int i, int a) { return kMMV[p][(i + 3) % 4][a]; }
constexpr int kMMB[3][3] = {{0, 0, -1}, {0, 1, 0}, {-1, 0, 0}};

constexpr int mm_cross_e_b(int p, int i, int a) {
    // (v x e_{i0})_a * 2 computed from the tables, for the static checks below
    return a == 0 ? kMMV[p][i][1] * mm_e2(p, i, 2) - kMMV[p][i][2] * mm_e2(p, i, 1)
         : a == 1 ? kMMV[p][i][2] * mm_e2(p, i, 0) - kMMV[p][i][0] * mm_e2(p, i, 2)
                  : kMMV[p][i][0] * mm_e2(p, i, 1) - kMMV[p][i][1] * mm_e2(p, i, 0);
}
constexpr bool mm_tables_consistent() {
    for (int p = 0; p < 3; ++p)
        for (int i = 0; i < 4; ++i) {
            int dot = 0;
            for (int a = 0; a < 3; ++a) {
                if (kMMV[p][(i + 2) % 4][a] != -kMMV[p][i][a]) return false;  // opposite pairs
                if (mm_cross_e_b(p, i, a) != 2 * kMMB[p][a]) return false;     // b = v x e
                dot += kMMV[p][i][a] * mm_e2(p, i, a);
            }
            if (dot != 0) return false;  // e perpendicular to v
        }
    return true;
}
static_assert(mm_tables_consistent(), "MM vector tables");

struct MM {
    static constexpr int Q = 50;
    static constexpr int kRestQ = 48;
    __host__ __device__ static constexpr int vel(int q, int a) {
        return q >= 48 ? 0 : kMMV[(q % 24) / 8][(q % 8) / 2][a];
    }
    __host__ __device__ static constexpr int opp(int q) {
        return q >= 48 ? q : (q / 8) * 8 + ((((q % 8) / 2) + 2) % 4) * 2 + (q % 2);
    }
};

// MM in difference form.  Of the MM populations only the differences
// d^{p(r)}_i = f^{p(r)}_{i0} - f^{p(r)}_{i1} enter D' and B (eq.
// MacroscopicFieldsMiller, with e_{i1} = -e_{i0} and b_{i1} = -b_{i0}), the two
// populations of a pair stream along the same v_i, and their equilibria
// (eq. equilibriumsMiller) differ by 2 u with u = (eps_r/4) E.e_{i0} +
// B.b_{i0}/(8 mu_r) (r = 0) or E.e_{i0}/4 + B.b_{i0}/8 (r = 1): the current
// term v.J/16 is common to both and cancels.  So d' = 4 u - d evolves on its
// own and reproduces E, B, D and H of the 50-population scheme exactly (up to
// rounding); only the charge density rho_c (the sums and rest populations)
// is not represented.  24 populations per cell instead of 50.
struct MMD {
    static constexpr int Q = 24;
    __host__ __device__ static constexpr int vel(int q, int a) { return kMMV[(q % 12) / 4][q % 4][a]; }
    __host__ __device__ static constexpr int opp(int q) { return (q / 12) * 12 + ((q % 12) / 4) * 4 + (q % 4 + 2) % 4; }
};

// ---------------------------------------------------------------- HV tables
// Section III velocity set: v1 = +x, v2 = +y, v3 = -x, v4 = -y, v5 = -z, v6 = +z.
constexpr int kHVV[6][3] = {{1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {0, 0, 1}};
constexpr int kHVOpp[6] = {2, 3, 0, 1, 5, 4};

struct HV {
    static constexpr int Q = 36;
    __host__ __device__ static constexpr int vel(int q, int a) { return kHVV[(q % 18) / 3][a]; }
    __host__ __device__ static constexpr int opp(int q) { return (q / 18) * 18 + kHVOpp[(q % 18) / 3] * 3 + q % 3; }
};

constexpr bool opp_consistent_mm() {
    for (int q = 0; q < MM::Q; ++q) {
        if (MM::opp(MM::opp(q)) != q) return false;
        for (int a = 0; a < 3; ++a)
            if (MM::vel(MM::opp(q), a) != -MM::vel(q, a)) return false;
    }
    return true;
}
constexpr bool opp_consistent_hv() {
    for (int q = 0; q < HV::Q; ++q) {
        if (HV::opp(HV::opp(q)) != q) return false;
        for (int a = 0; a < 3; ++a)
            if (HV::vel(HV::opp(q), a) != -HV::vel(q, a)) return false;
    }
    return true;
}
constexpr bool opp_consistent_mmd() {
    for (int q = 0; q < MMD::Q; ++q) {
        if (MMD::opp(MMD::opp(q)) != q) return false;
        for (int a = 0; a < 3; ++a)
            if (MMD::vel(MMD::opp(q), a) != -MMD::vel(q, a)) return false;
    }
    return true;
}
static_assert(opp_consistent_mm() && opp_consistent_hv() && opp_consistent_mmd(), "opposite-direction maps");

// ---------------------------------------------------------------- per cell
// x / d given inv = 1 / d (rounded): one Newton correction of the product makes
// the quotient (nearly always) the correctly rounded one.  Multiplying by a
// rounded reciprocal alone biases every update the same way, and over 10^4
// steps that bias accumulates linearly into phase drift; rounding that is
// unbiased only accumulates as a random walk.
__device__ __forceinline__ float div_rn(float x, float d, float inv) {
    const float q = x * inv;
    const float r = __builtin_fmaf(-q, d, x);
    return __builtin_fmaf(r, inv, q);
}

// Media and source seen by one cell at one step.
struct CellMedia {
    float eps_r, mu_r, sigma;
};

// Reported fields of one cell (pre-collision state).
struct CellFields {
    float E[3], B[3], D[3], H[3];
};

// MM collision (Section II): moments (eq. MacroscopicFieldsMiller), physical E
// and current with both an ohmic and a prescribed part
//   E = (D'/eps_r - mu0 Jsrc / (4 eps_r)) / (1 + mu0 sigma / (4 eps_r)),
//   J = sigma E + Jsrc,                 (mu0 = 2)
// equilibria (eq. equilibriumsMiller) and f' = 2 f_eq - f (eq. CollisionMiller,
// applied to both rest populations).  f is overwritten with f'.
__device__ __forceinline__ void mm_collide(float (&f)[50], const CellMedia &m, const float Js[3], CellFields &o) {
    float D[3] = {0.f, 0.f, 0.f}, B[3] = {0.f, 0.f, 0.f};
    float rho = f[48];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float sb = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float d0 = f[p * 8 + i * 2] - f[p * 8 + i * 2 + 1];        // f_{i0} - f_{i1}, r = 0
            const float d1 = f[24 + p * 8 + i * 2] - f[24 + p * 8 + i * 2 + 1];  // r = 1
            rho += f[p * 8 + i * 2] + f[p * 8 + i * 2 + 1];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (mm_e2(p, i, a) != 0) D[a] += (mm_e2(p, i, a) > 0 ? 0.5f : -0.5f) * d0;
            sb += d1;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (kMMB[p][a] != 0) B[a] += kMMB[p][a] > 0 ? sb : -sb;
    }
    // mu0 / 4 = 1/2:  E = (D' - Jsrc / 2) / (eps_r + sigma / 2)
    const float den = m.eps_r + 0.5f * m.sigma;
    const float inv = 1.0f / den;
    float E[3], J[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        E[a] = div_rn(D[a] - 0.5f * Js[a], den, inv);
        J[a] = m.sigma * E[a] + Js[a];
        o.E[a] = E[a];
        o.B[a] = B[a];
        o.D[a] = m.eps_r * E[a];
        o.H[a] = 0.5f * (B[a] / m.mu_r);
    }
    const float ke0 = 0.25f * m.eps_r, imu = 1.0f / m.mu_r;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float bb = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (kMMB[p][a] != 0) bb += kMMB[p][a] > 0 ? B[a] : -B[a];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float vj = 0.f, ee = 0.f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (kMMV[p][i][a] != 0) vj += kMMV[p][i][a] > 0 ? J[a] : -J[a];
                if (mm_e2(p, i, a) != 0) ee += mm_e2(p, i, a) > 0 ? E[a] : -E[a];
            }
            ee *= 0.5f;                     // E . e_{i0}
            const float a0 = vj * 0.0625f;  // v . J / 16
            const float u0 = ke0 * ee + 0.125f * div_rn(bb, m.mu_r, imu);
            const float u1 = 0.25f * ee + 0.125f * bb;
            const int q0 = p * 8 + i * 2, q1 = 24 + p * 8 + i * 2;
            f[q0] = 2.f * (a0 + u0) - f[q0];
            f[q0 + 1] = 2.f * (a0 - u0) - f[q0 + 1];
            f[q1] = 2.f * (a0 + u1) - f[q1];
            f[q1 + 1] = 2.f * (a0 - u1) - f[q1 + 1];
        }
    }
    f[48] = 2.f * rho - f[48];
    f[49] = 2.f * rho - f[49];
}

// MM equilibrium of given E, B with J = 0 and rho_c = 0 (initialisation and
// hard sources).
__device__ __forceinline__ void mm_field_equilibrium(float (&f)[50], const CellMedia &m, const float E[3],
                                                     const float B[3]) {
    const float ke0 = 0.25f * m.eps_r, imu = 1.0f / m.mu_r;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float bb = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (kMMB[p][a] != 0) bb += kMMB[p][a] > 0 ? B[a] : -B[a];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float ee = 0.f;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (mm_e2(p, i, a) != 0) ee += mm_e2(p, i, a) > 0 ? E[a] : -E[a];
            ee *= 0.5f;
            const float u0 = ke0 * ee + 0.125f * div_rn(bb, m.mu_r, imu);
            const float u1 = 0.25f * ee + 0.125f * bb;
            const int q0 = p * 8 + i * 2, q1 = 24 + p * 8 + i * 2;
            f[q0] = u0;
            f[q0 + 1] = -u0;
            f[q1] = u1;
            f[q1 + 1] = -u1;
        }
    }
    f[48] = 0.f;
    f[49] = 0.f;
}

// MM in difference form: the same moments, constitutive relations and u as
// mm_collide, with d' = 4 u - d (see MMD).
__device__ __forceinline__ void mmd_collide(float (&d)[24], const CellMedia &m, const float Js[3], CellFields &o) {
    float D[3] = {0.f, 0.f, 0.f}, B[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float sb = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float d0 = d[p * 4 + i], d1 = d[12 + p * 4 + i];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (mm_e2(p, i, a) != 0) D[a] += (mm_e2(p, i, a) > 0 ? 0.5f : -0.5f) * d0;
            sb += d1;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (kMMB[p][a] != 0) B[a] += kMMB[p][a] > 0 ? sb : -sb;
    }
    const float den = m.eps_r + 0.5f * m.sigma;
    const float inv = 1.0f / den;
    float E[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        E[a] = div_rn(D[a] - 0.5f * Js[a], den, inv);
        o.E[a] = E[a];
        o.B[a] = B[a];
        o.D[a] = m.eps_r * E[a];
        o.H[a] = 0.5f * (B[a] / m.mu_r);
    }
    const float ke0 = 0.25f * m.eps_r, imu = 1.0f / m.mu_r;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float bb = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (kMMB[p][a] != 0) bb += kMMB[p][a] > 0 ? B[a] : -B[a];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float ee = 0.f;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (mm_e2(p, i, a) != 0) ee += mm_e2(p, i, a) > 0 ? E[a] : -E[a];
            ee *= 0.5f;
            const float u0 = ke0 * ee + 0.125f * div_rn(bb, m.mu_r, imu);
            const float u1 = 0.25f * ee + 0.125f * bb;
            d[p * 4 + i] = 4.f * u0 - d[p * 4 + i];
            d[12 + p * 4 + i] = 4.f * u1 - d[12 + p * 4 + i];
        }
    }
}

// d of the MM equilibrium of given E, B (J = 0): 2 u.
__device__ __forceinline__ void mmd_field_equilibrium(float (&d)[24], const CellMedia &m, const float E[3],
                                                      const float B[3]) {
    const float ke0 = 0.25f * m.eps_r, imu = 1.0f / m.mu_r;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float bb = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (kMMB[p][a] != 0) bb += kMMB[p][a] > 0 ? B[a] : -B[a];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float ee = 0.f;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (mm_e2(p, i, a) != 0) ee += mm_e2(p, i, a) > 0 ? E[a] : -E[a];
            ee *= 0.5f;
            d[p * 4 + i] = 2.f * (ke0 * ee + 0.125f * div_rn(bb, m.mu_r, imu));
            d[12 + p * 4 + i] = 2.f * (0.25f * ee + 0.125f * bb);
        }
    }
}

// HV lattice constants: eps0 = mu0 = 3 (vacuum speed 1/3, impedance 1).
constexpr float kHVEps0 = 3.0f, kHVMu0 = 3.0f;

// cross product of an axis velocity with a vector, component a
template <int I>
__device__ __forceinline__ float hv_vcross(const float w[3], int a) {
    constexpr int vx = kHVV[I][0], vy = kHVV[I][1], vz = kHVV[I][2];
    return a == 0 ? vy * w[2] - vz * w[1] : a == 1 ? vz * w[0] - vx * w[2] : vx * w[1] - vy * w[0];
}

template <int I>
__device__ __forceinline__ void hv_collide_dir(float (&f)[36], const float D[3], const float B[3], const float E[3],
                                               const float H[3], const float J[3]) {
    constexpr int vx = kHVV[I][0], vy = kHVV[I][1], vz = kHVV[I][2];
    const float Jv = vx * J[0] + vy * J[1] + vz * J[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int va = a == 0 ? vx : a == 1 ? vy : vz;
        const int qe = I * 3 + a, qh = 18 + I * 3 + a;
        // e' = 2 e_eq - e + T,  e_eq = (D - 3 v x H) / 6,  T = -(J.v) v / 2
        const float ee = div_rn(D[a] - 3.f * hv_vcross<I>(H, a), 6.f, 1.f / 6.f);
        f[qe] = 2.f * ee - f[qe] - 0.5f * Jv * va;
        // h' = 2 h_eq - h,  h_eq = (B + 3 v x E) / 6
        const float he = div_rn(B[a] + 3.f * hv_vcross<I>(E, a), 6.f, 1.f / 6.f);
        f[qh] = 2.f * he - f[qh];
    }
}

// Modified HV collision (Section III): D = sum e_i, B = sum h_i (eq.
// MacroscopicFieldsHV), E = D / eps, H = B / mu, J = sigma E + Jsrc, equilibria
// of eq. (equilibriumHV), e' = 2 e_eq - e + T (eq. CollisionmodifiedHV),
// h' = 2 h_eq - h.
__device__ __forceinline__ void hv_collide(float (&f)[36], const CellMedia &m, const float Js[3], CellFields &o) {
    float D[3], B[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        D[a] = ((f[a] + f[3 + a]) + (f[6 + a] + f[9 + a])) + (f[12 + a] + f[15 + a]);
        B[a] = ((f[18 + a] + f[21 + a]) + (f[24 + a] + f[27 + a])) + (f[30 + a] + f[33 + a]);
    }
    const float eps = kHVEps0 * m.eps_r, mu = kHVMu0 * m.mu_r;
    const float ie = 1.0f / eps, im = 1.0f / mu;
    float E[3], H[3], J[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        E[a] = div_rn(D[a], eps, ie);
        H[a] = div_rn(B[a], mu, im);
        J[a] = m.sigma * E[a] + Js[a];
        o.E[a] = E[a];
        o.B[a] = B[a];
        o.D[a] = D[a];
        o.H[a] = H[a];
    }
    hv_collide_dir<0>(f, D, B, E, H, J);
    hv_collide_dir<1>(f, D, B, E, H, J);
    hv_collide_dir<2>(f, D, B, E, H, J);
    hv_collide_dir<3>(f, D, B, E, H, J);
    hv_collide_dir<4>(f, D, B, E, H, J);
    hv_collide_dir<5>(f, D, B, E, H, J);
}

template <int I>
__device__ __forceinline__ void hv_eq_dir(float (&f)[36], const float D[3], const float B[3], const float E[3],
                                          const float H[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f[I * 3 + a] = div_rn(D[a] - 3.f * hv_vcross<I>(H, a), 6.f, 1.f / 6.f);
        f[18 + I * 3 + a] = div_rn(B[a] + 3.f * hv_vcross<I>(E, a), 6.f, 1.f / 6.f);
    }
}

// HV equilibrium of given E, B (D = eps E, H = B / mu).
__device__ __forceinline__ void hv_field_equilibrium(float (&f)[36], const CellMedia &m, const float E[3],
                                                     const float B[3]) {
    const float eps = kHVEps0 * m.eps_r, mu = kHVMu0 * m.mu_r;
    const float im = 1.0f / mu;
    float D[3], H[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        D[a] = eps * E[a];
        H[a] = div_rn(B[a], mu, im);
    }
    hv_eq_dir<0>(f, D, B, E, H);
    hv_eq_dir<1>(f, D, B, E, H);
    hv_eq_dir<2>(f, D, B, E, H);
    hv_eq_dir<3>(f, D, B, E, H);
    hv_eq_dir<4>(f, D, B, E, H);
    hv_eq_dir<5>(f, D, B, E, H);
}

// ---------------------------------------------------------------- shift
// Equilibrium-shifted 16-bit storage.  A population leaving cell x is stored
// as g_q = f'_q - phi_q(R_x), where R_x is a per-cell record of the emitting
// cell (E, B, eps_r, 1/mu_r, each rounded to BF16) and phi_q(R) is the
// field part of the equilibrium of q for that record (the current term
// v.J/16 of MM and the HV source term are left out, and the rest populations
// are not shifted).  Since f' = 2 f_eq - f, f'_q - f_eq_q = f_eq_q - f_q is the
// non-equilibrium part, typically a small fraction of f_q on smooth fields, so
// the 16-bit rounding error shrinks by that fraction.  The reader of
// population q at x adds phi_q(R_{x - v_q}) back, evaluated by the same code
// on the same rounded record.
//
// Record layout: 8 BF16 values, rec[0..2] = E, rec[3..5] = B, rec[6] = eps_r,
// rec[7] = 1 / mu_r (16 bytes, one aligned vector access).
struct Rec {
    float E[3], B[3], eps, imu;
};
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Two floats rounded to BF16 (nearest, ties to even) in one 32-bit word, low
// half first: one v_cvt_pk_bf16_f32 on gfx950.
__device__ __forceinline__ uint32_t bf16x2_rn(float lo, float hi) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    const f2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, b2));
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

__device__ __forceinline__ Rec rec_unpack(u32x4 u) {
    Rec r;
    r.E[0] = bf16_lo(u.x);
    r.E[1] = bf16_hi(u.x);
    r.E[2] = bf16_lo(u.y);
    r.B[0] = bf16_hi(u.y);
    r.B[1] = bf16_lo(u.z);
    r.B[2] = bf16_hi(u.z);
    r.eps = bf16_lo(u.w);
    r.imu = bf16_hi(u.w);
    return r;
}

// Round a record to BF16; returns the packed 16 bytes and (in r) the rounded
// values, exactly as rec_unpack will read them back.
__device__ __forceinline__ u32x4 rec_pack(const float E[3], const float B[3], float eps, float imu, Rec &r) {
    u32x4 u;
    u.x = bf16x2_rn(E[0], E[1]);
    u.y = bf16x2_rn(E[2], B[0]);
    u.z = bf16x2_rn(B[1], B[2]);
    u.w = bf16x2_rn(eps, imu);
    r = rec_unpack(u);
    return u;
}

// Per model: the distinct moving velocities k (every shifted population
// belongs to exactly one), phi<k>(R, s, u): the kNPhi distinct values of
// s * phi_q(R) over the populations q of k, and apply<k>(f, u): f_q += those
// values.  MM's and the difference form's products and sums are written out
// with explicit FMAs, so that a value computed by one thread and handed to
// another (the row form's record exchange) has the same bits as one computed
// and applied in place.
template <class M>
struct Shift;
template <>
struct Shift<MM> {
    static constexpr int kNV = 12;    // k = p * 4 + i; populations 2k, 2k+1, 24+2k, 24+2k+1
    static constexpr int kNPhi = 2;   // +-u0 (electric pair), +-u1 (magnetic pair)
    __host__ __device__ static constexpr int vel(int k, int a) { return kMMV[k / 4][k % 4][a]; }
    template <int K>
    __device__ static void phi(const Rec &r, float s, float (&u)[kNPhi]) {
        constexpr int p = K / 4, i = K % 4;
        float ee = 0.f, bb = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (mm_e2(p, i, a) != 0) ee += mm_e2(p, i, a) > 0 ? r.E[a] : -r.E[a];
            if (kMMB[p][a] != 0) bb += kMMB[p][a] > 0 ? r.B[a] : -r.B[a];
        }
        // E.e_{i0} = ee / 2; f0_eq = eps/4 E.e + B.b/(8 mu), f1_eq = E.e/4 + B.b/8
        u[0] = s * __builtin_fmaf(0.125f * r.eps, ee, (0.125f * r.imu) * bb);
        u[1] = s * (0.125f * ee + 0.125f * bb);  // both products exact
    }
    template <int K>
    __device__ static void apply(float (&f)[50], const float (&u)[kNPhi]) {
        f[2 * K] += u[0];
        f[2 * K + 1] -= u[0];
        f[24 + 2 * K] += u[1];
        f[24 + 2 * K + 1] -= u[1];
    }
};
template <>
struct Shift<MMD> {
    static constexpr int kNV = 12;  // k = p * 4 + i; populations k, 12 + k
    static constexpr int kNPhi = 2;
    __host__ __device__ static constexpr int vel(int k, int a) { return kMMV[k / 4][k % 4][a]; }
    template <int K>
    __device__ static void phi(const Rec &r, float s, float (&u)[kNPhi]) {
        constexpr int p = K / 4, i = K % 4;
        float ee = 0.f, bb = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (mm_e2(p, i, a) != 0) ee += mm_e2(p, i, a) > 0 ? r.E[a] : -r.E[a];
            if (kMMB[p][a] != 0) bb += kMMB[p][a] > 0 ? r.B[a] : -r.B[a];
        }
        // d = 2 u (see Shift<MM>)
        u[0] = s * __builtin_fmaf(0.25f * r.eps, ee, (0.25f * r.imu) * bb);
        u[1] = s * (0.25f * ee + 0.25f * bb);
    }
    template <int K>
    __device__ static void apply(float (&f)[24], const float (&u)[kNPhi]) {
        f[K] += u[0];
        f[12 + K] += u[1];
    }
};
template <>
struct Shift<HV> {
    static constexpr int kNV = 6;    // k = i; populations 3i + a, 18 + 3i + a
    static constexpr int kNPhi = 6;  // e_a, h_a
    __host__ __device__ static constexpr int vel(int k, int a) { return kHVV[k][a]; }
    // (HV's phi never passes between threads, so the compiler may contract it)
    template <int K>
    __device__ static void phi(const Rec &r, float s, float (&u)[kNPhi]) {
        // e_eq = (3 eps_r E - v x B / mu_r) / 6,  h_eq = (B + 3 v x E) / 6
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u[a] = s * (0.5f * r.eps * r.E[a] - (1.f / 6.f) * r.imu * hv_vcross<K>(r.B, a));
            u[3 + a] = s * ((1.f / 6.f) * r.B[a] + 0.5f * hv_vcross<K>(r.E, a));
        }
    }
    template <int K>
    __device__ static void apply(float (&f)[36], const float (&u)[kNPhi]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            f[3 * K + a] += u[a];
            f[18 + 3 * K + a] += u[3 + a];
        }
    }
};

// f += s * phi(R_k) for every velocity k, with R_k produced by rec_of(k).
template <class M, int K = 0, class F>
__device__ __forceinline__ void shift_all(float (&f)[M::Q], float s, F &&rec_of) {
    if constexpr (K < Shift<M>::kNV) {
        float u[Shift<M>::kNPhi];
        Shift<M>::template phi<K>(rec_of(K), s, u);
        Shift<M>::template apply<K>(f, u);
        shift_all<M, K + 1>(f, s, rec_of);
    }
}

// model dispatch
template <class M>
struct Cell;
template <>
struct Cell<MM> {
    __device__ static void collide(float (&f)[50], const CellMedia &m, const float Js[3], CellFields &o) {
        mm_collide(f, m, Js, o);
    }
    __device__ static void equilibrium(float (&f)[50], const CellMedia &m, const float E[3], const float B[3]) {
        mm_field_equilibrium(f, m, E, B);
    }
};
template <>
struct Cell<MMD> {
    __device__ static void collide(float (&f)[24], const CellMedia &m, const float Js[3], CellFields &o) {
        mmd_collide(f, m, Js, o);
    }
    __device__ static void equilibrium(float (&f)[24], const CellMedia &m, const float E[3], const float B[3]) {
        mmd_field_equilibrium(f, m, E, B);
    }
};
template <>
struct Cell<HV> {
    __device__ static void collide(float (&f)[36], const CellMedia &m, const float Js[3], CellFields &o) {
        hv_collide(f, m, Js, o);
    }
    __device__ static void equilibrium(float (&f)[36], const CellMedia &m, const float E[3], const float B[3]) {
        hv_field_equilibrium(f, m, E, B);
    }
};

}  // namespace lbem
