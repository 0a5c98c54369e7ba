// media.h -- index distributions n(P) and grad n(P) on the device.
//
// Two evaluators per medium:
//   med64<K>  double precision n and grad n (plain march, surface events and
//             the near-grazing decisions of the single-precision march).  Each
//             formula is evaluated in the order it is written (n, then the
//             gradient by the chain rule), with divisions kept as divisions,
//             so that with FMA contraction disabled the results are the
//             correctly rounded steps of the textbook expressions;
//   med32<K>  single precision n and grad n at P_i plus the index difference
//             dn = n(P_i) - n(P_{i-1}) along the last move s = P_i - P_{i-1},
//             computed from s directly instead of as the difference of two
//             rounded indices.  The vectorial law only needs mu_i - 1 =
//             -dn / n_i (Eqs. (9)-(10), (19)); near isoindicial turning points
//             dn is ~1e-8 while a rounded index carries ~1e-7 of error, so the
//             difference form is what keeps the single-precision march on the
//             same side of every refraction/TIR decision as a double one.
//
// Parameter storage (MediumDev.q, raw as given to vrt_medium_create_analytic):
//   HOMOGENEOUS [n]  LINEAR [n0, gx, gy, gz]  LUNEBURG [R, cx, cy, cz]
//   FIBER [n_c, Delta, R, cx, cy]  GAUSSIAN [n0] + bumps_d (A, sigma, cx, cy, cz) x K
//   SPHERICAL [a0, a1, a2, a3, cx, cy, cz]  N2P [R, F, beta, gamma]
//   ZERNIKE [n0, dn, rho_max, z_max] + bumps_d = c[j - 1][l] (16 x 4, row j - 1 of
//           Fringe term j, column l of Legendre polynomial l), K = mask of the
//           rows that hold a nonzero coefficient
// MedF.q holds single-precision derived constants (see vrt_api.hip).
// Discretized media keep the node values and node records
// (n, h_x, h_y, h_z) where h_a is the central difference of the node values
// along axis a divided by the number of node spacings it spans (2, or 1 at
// the first/last node): exact in float for nearby values; grad n = h * inv_h.
#pragma once

#include <type_traits>

#include "vrt_common.h"

namespace vrt {

// ---------------------------------------------------------------------------
// double precision
// ---------------------------------------------------------------------------
__device__ __forceinline__ double grid_node64(const MediumDev &m, int i, int j, int k) {
    return (double)m.grid[((size_t)k * m.ny + j) * m.nx + i];
}

// node central difference along axis a (one-sided at the first/last node)
__device__ inline double grid_cdiff64(const MediumDev &m, int i, int j, int k, int a) {
    const int nn = a == 0 ? m.nx : (a == 1 ? m.ny : m.nz);
    const int idx = a == 0 ? i : (a == 1 ? j : k);
    int lo = idx, hi = idx;
    double span;
    if (idx == 0) {
        hi = 1;
        span = m.h[a];
    } else if (idx == nn - 1) {
        lo = nn - 2;
        span = m.h[a];
    } else {
        lo = idx - 1;
        hi = idx + 1;
        span = 2.0 * m.h[a];
    }
    const double vh = a == 0 ? grid_node64(m, hi, j, k)
                             : (a == 1 ? grid_node64(m, i, hi, k) : grid_node64(m, i, j, hi));
    const double vl = a == 0 ? grid_node64(m, lo, j, k)
                             : (a == 1 ? grid_node64(m, i, lo, k) : grid_node64(m, i, j, lo));
    return (vh - vl) / span;
}

__device__ inline void grid_cell64(const MediumDev &m, d3 P, int c[3], double f[3]) {
    const int nn[3] = {m.nx, m.ny, m.nz};
    for (int a = 0; a < 3; ++a) {
        double x = get(P, a);
        x = x < m.lo[a] ? m.lo[a] : (x > m.hi[a] ? m.hi[a] : x);
        const double u = (x - m.lo[a]) / m.h[a];
        int ci = (int)floor(u);
        ci = ci < 0 ? 0 : (ci > nn[a] - 2 ? nn[a] - 2 : ci);
        c[a] = ci;
        f[a] = u - (double)ci;
    }
}

// Fringe Zernike polynomial j (1..16, unnormalised) at (u, v) in Cartesian form,
// with its partial derivatives.  r2 = u^2 + v^2.
__device__ __forceinline__ void fringe64(int j, double u, double v, double &Z, double &Zu,
                                         double &Zv) {
    const double r2 = u * u + v * v;
    switch (j) {
    case 1: Z = 1.0; Zu = 0.0; Zv = 0.0; break;
    case 2: Z = u; Zu = 1.0; Zv = 0.0; break;
    case 3: Z = v; Zu = 0.0; Zv = 1.0; break;
    case 4: Z = 2.0 * r2 - 1.0; Zu = 4.0 * u; Zv = 4.0 * v; break;
    case 5: Z = u * u - v * v; Zu = 2.0 * u; Zv = -2.0 * v; break;
    case 6: Z = 2.0 * u * v; Zu = 2.0 * v; Zv = 2.0 * u; break;
    case 7: Z = (3.0 * r2 - 2.0) * u; Zu = 3.0 * r2 - 2.0 + 6.0 * u * u; Zv = 6.0 * u * v; break;
    case 8: Z = (3.0 * r2 - 2.0) * v; Zu = 6.0 * u * v; Zv = 3.0 * r2 - 2.0 + 6.0 * v * v; break;
    case 9: {
        Z = (6.0 * r2 - 6.0) * r2 + 1.0;
        const double d = 24.0 * r2 - 12.0;  // dZ/du = d u
        Zu = d * u;
        Zv = d * v;
        break;
    }
    case 10: Z = u * u * u - 3.0 * u * v * v; Zu = 3.0 * (u * u - v * v); Zv = -6.0 * u * v; break;
    case 11: Z = 3.0 * u * u * v - v * v * v; Zu = 6.0 * u * v; Zv = 3.0 * (u * u - v * v); break;
    case 12: {
        const double a = 4.0 * r2 - 3.0, b = u * u - v * v;
        Z = a * b;
        Zu = 8.0 * u * b + 2.0 * a * u;
        Zv = 8.0 * v * b - 2.0 * a * v;
        break;
    }
    case 13: {
        const double a = 4.0 * r2 - 3.0, b = 2.0 * u * v;
        Z = a * b;
        Zu = 8.0 * u * b + 2.0 * a * v;
        Zv = 8.0 * v * b + 2.0 * a * u;
        break;
    }
    case 14: case 15: {
        const double a = (10.0 * r2 - 12.0) * r2 + 3.0, da = 40.0 * r2 - 24.0;  // da = 2 a'(r2)
        const double t = j == 14 ? u : v;
        Z = a * t;
        Zu = da * u * t + (j == 14 ? a : 0.0);
        Zv = da * v * t + (j == 15 ? a : 0.0);
        break;
    }
    default: {  // 16
        Z = ((20.0 * r2 - 30.0) * r2 + 12.0) * r2 - 1.0;
        const double d = (120.0 * r2 - 120.0) * r2 + 24.0;  // 2 dZ/d(r2)
        Zu = d * u;
        Zv = d * v;
        break;
    }
    }
}

template <int MK>
__device__ inline void med64(const MediumDev &m, d3 P, double &n, d3 &g) {
    const double *p = m.q;
    if constexpr (MK == VRT_MEDIUM_HOMOGENEOUS) {
        n = p[0];
        g = mk(0, 0, 0);
    } else if constexpr (MK == VRT_MEDIUM_LINEAR) {
        n = p[0] + p[1] * P.x + p[2] * P.y + p[3] * P.z;
        g = mk(p[1], p[2], p[3]);
    } else if constexpr (MK == VRT_MEDIUM_LUNEBURG) {
        // n = sqrt(2 - r^2/R^2), grad n = -(P - C) / (R^2 n)
        const double R = p[0];
        const d3 o = P - mk(p[1], p[2], p[3]);
        n = sqrt(2.0 - dot(o, o) / (R * R));
        g = mk(-o.x / (R * R * n), -o.y / (R * R * n), -o.z / (R * R * n));
    } else if constexpr (MK == VRT_MEDIUM_FIBER) {
        // Sec. IV, Eq. (21): core n^2 = n_c^2 (1 - 2 Delta rho^2 / R^2); cladding constant
        const double nc = p[0], Dl = p[1], R = p[2];
        const double x = P.x - p[3], y = P.y - p[4];
        const double r2 = x * x + y * y;
        if (r2 <= R * R) {
            n = nc * sqrt(1.0 - 2.0 * Dl * r2 / (R * R));
            const double k = -2.0 * Dl * nc * nc / (R * R * n);
            g = mk(k * x, k * y, 0.0);
        } else {
            n = nc * sqrt(1.0 - 2.0 * Dl);
            g = mk(0, 0, 0);
        }
    } else if constexpr (MK == VRT_MEDIUM_GAUSSIAN) {
        // n = n0 + sum A exp(-|P - c|^2 / (2 sigma^2)), grad = -sum A e (P - c) / sigma^2
        n = p[0];
        g = mk(0, 0, 0);
        for (int k = 0; k < m.K; ++k) {
            const double *b = m.bumps_d + 5 * k;
            const double A = b[0], s = b[1];
            const d3 o = P - mk(b[2], b[3], b[4]);
            const double e = A * exp(-dot(o, o) / (2.0 * s * s));
            n += e;
            g.x += -e * o.x / (s * s);
            g.y += -e * o.y / (s * s);
            g.z += -e * o.z / (s * s);
        }
    } else if constexpr (MK == VRT_MEDIUM_SPHERICAL) {
        // Sec. V, Eq. (26) in Cartesian form about the centre: with c = cos(theta) = z/r,
        // G1 = 0.3 (r^2 - 1), G2 = r cos(5 theta) = z (16 c^4 - 20 c^2 + 5) (Chebyshev T5),
        // G3 = r^2 sin^2(theta) cos(2 phi) = x^2 - y^2.  G2 is homogeneous of degree 1:
        // its gradient is bounded but has no limit at r = 0 (returned as NaN: case (ii)).
        const double a0 = p[0], a1 = p[1], a2 = p[2], a3 = p[3];
        const double x = P.x - p[4], y = P.y - p[5], z = P.z - p[6];
        const double r2 = x * x + y * y + z * z;
        if (r2 == 0.0) {
            n = a0 - 0.3 * a1;
            g = mk(NAN, NAN, NAN);
        } else {
            const double c2 = z * z / r2;
            n = a0 + a1 * (0.3 * (r2 - 1.0)) + a2 * (z * ((16.0 * c2 - 20.0) * c2 + 5.0)) +
                a3 * (x * x - y * y);
            const double h = z * c2 / r2 * (40.0 - 64.0 * c2);  // d G2/dx = h x, d G2/dy = h y
            const double gz2 = ((-64.0 * c2 + 120.0) * c2 - 60.0) * c2 + 5.0;
            g = mk(a1 * (0.6 * x) + a2 * (h * x) + a3 * (2.0 * x),
                   a1 * (0.6 * y) + a2 * (h * y) - a3 * (2.0 * y), a1 * (0.6 * z) + a2 * gz2);
        }
    } else if constexpr (MK == VRT_MEDIUM_N2P) {
        // Sec. VI, Eq. (27): n = u^gamma, u = 1 + w^beta, w = (R^2 - rho^2/4) / F^2 about the
        // z axis; grad n = 2 dn/d(rho^2) (x, y, 0) with
        // dn/d(rho^2) = gamma u^(gamma-1) beta w^(beta-1) (-1 / (4 F^2)).
        const double R = p[0], F = p[1], be = p[2], ga = p[3];
        const double rho2 = P.x * P.x + P.y * P.y;
        const double w = (R * R - rho2 / 4.0) / (F * F);
        const double wb = pow(w, be);
        const double u = 1.0 + wb;
        n = pow(u, ga);
        const double k = 2.0 * (ga * (n / u) * be * (wb / w) * (-1.0 / (4.0 * F * F)));
        g = mk(k * P.x, k * P.y, 0.0);
    } else if constexpr (MK == VRT_MEDIUM_ZERNIKE) {
        // Sec. V: n = n0 + dn sum_j Z_j(u, v) A_j(w) with u = x / rho_max,
        // v = y / rho_max, w = 2 z / z_max - 1 and A_j(w) = sum_l c[j][l] P_l(w)
        // (Legendre P0..P3); the chain rule scales d/du, d/dv by 1 / rho_max and
        // d/dw by 2 / z_max.
        const double n0 = p[0], dn = p[1], rm = p[2], zm = p[3];
        const double u = P.x / rm, v = P.y / rm, w = 2.0 * P.z / zm - 1.0;
        const double L1 = w, L2 = (3.0 * w * w - 1.0) / 2.0, L3 = (5.0 * w * w - 3.0) * w / 2.0;
        const double dL2 = 3.0 * w, dL3 = (15.0 * w * w - 3.0) / 2.0;
        double s = 0.0, su = 0.0, sv = 0.0, sw = 0.0;
#pragma unroll
        for (int j = 1; j <= 16; ++j) {  // unrolled: each term's form is fixed at compile time
            if (!((m.K >> (j - 1)) & 1)) continue;
            const double *c = m.bumps_d + 4 * (j - 1);
            const double A = c[0] + c[1] * L1 + c[2] * L2 + c[3] * L3;
            const double dA = c[1] + c[2] * dL2 + c[3] * dL3;
            double Z, Zu, Zv;
            fringe64(j, u, v, Z, Zu, Zv);
            s += Z * A;
            su += Zu * A;
            sv += Zv * A;
            sw += Z * dA;
        }
        n = n0 + dn * s;
        g = mk(dn * su / rm, dn * sv / rm, dn * sw * 2.0 / zm);
    } else {  // GRID: trilinear n, trilinear node central differences
        int c[3];
        double f[3];
        grid_cell64(m, P, c, f);
        n = 0.0;
        g = mk(0, 0, 0);
        if (m.rec_exact) {
            // the node records hold each value and its differences over the
            // spacings exactly, so (double)h_a / h equals (v_hi - v_lo) / span:
            // one 16-byte load per corner instead of seven scattered ones
            const size_t sy = (size_t)m.nx, sz = (size_t)m.nx * m.ny;
            const size_t o = (size_t)c[2] * sz + (size_t)c[1] * sy + c[0];
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                                         (dz ? f[2] : 1.0 - f[2]);
                        const float4 r = m.rec[o + dx + dy * sy + dz * sz];
                        n += w * (double)r.x;
                        g.x += w * ((double)r.y / m.h[0]);
                        g.y += w * ((double)r.z / m.h[1]);
                        g.z += w * ((double)r.w / m.h[2]);
                    }
            return;
        }
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                                     (dz ? f[2] : 1.0 - f[2]);
                    const int i = c[0] + dx, j = c[1] + dy, k = c[2] + dz;
                    n += w * grid_node64(m, i, j, k);
                    g.x += w * grid_cdiff64(m, i, j, k, 0);
                    g.y += w * grid_cdiff64(m, i, j, k, 1);
                    g.z += w * grid_cdiff64(m, i, j, k, 2);
                }
    }
}

template <int MK>
__device__ __forceinline__ double index64(const MediumDev &m, d3 P) {
    double n;
    d3 g;
    med64<MK>(m, P, n, g);
    return n;
}

// ---------------------------------------------------------------------------
// single precision with the index difference along the last move
// ---------------------------------------------------------------------------
struct MedF {  // single-precision constants of the analytic media
    float q[8];
};

// Accuracy of the truncated expm1 in the Gaussian index difference.  The
// argument is the change of a bump exponent over one step,
// dq = ((P - c).s - |s|^2/2) / sigma^2; with t = |P - c| / sigma and
// rho = Delta / sigma, |dq| <= t rho (+ rho^2 / 2).  Dropping the terms from
// x^(d+1) on costs at most |A| exp(-t^2/2) (t rho)^(d+1) / (d+1)! in
// n_i - n_{i-1}, largest at t = sqrt(d+1).  Degree 3 is used while
// rho <= kGaussRho3 (error < 3e-11 |A| per bump at rho = 8e-3), degree 5 up
// to kGaussRhoMax (error < 2e-11 |A| at rho = 0.05); longer steps are refused
// for the single-precision path.  rho is bounded per trace by
// dL0 / (n_min sigma_min), n_min = n0 - sum |A|.
constexpr double kGaussRho3 = 8e-3;
constexpr double kGaussRhoMax = 5e-2;

// Single-precision reciprocal and square root from the hardware
// approximations (~1 ulp); the march needs no correctly rounded results in
// its float part (step lengths, gamma, normals).
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Media whose index the single-precision march takes in double (their terms
// span several orders of magnitude or need pow): the march evaluates med64 at
// the compensated position once per step and keeps n(P_{i-1}) in double, so
// the index difference is the difference of two double indices (lane32.h).
template <int MK>
constexpr bool kIndexIn64 =
    MK == VRT_MEDIUM_SPHERICAL || MK == VRT_MEDIUM_N2P || MK == VRT_MEDIUM_ZERNIKE;

// P: point P_i, s = P_i - P_{i-1}, n_last = n(P_{i-1}).  n + nl is the index
// at P_i where the medium's constant part is split off (homogeneous, linear,
// Gaussian: n0 exactly as given plus the float-summed variable part); nl = 0
// for the Luneburg and fiber media.  bumps: the Gaussian
// table (m.bumps_f) -- a restrict kernel argument in the batch kernel, a
// constant-address-space pointer in the serving kernel; its loads are scalar
// in both.
// MedF.q: HOMOGENEOUS [n, n - (float)n]; LINEAR [n0, gx, gy, gz, n0 - (float)n0];
// LUNEBURG [., cx, cy, cz, 1/R^2]; FIBER [n_c, Delta, ., cx, cy, 2 Delta n_c^2/R^2,
// n_clad, R^2]; GAUSSIAN [n0, largest dL0 for the degree-3 difference form,
// n0 - (float)n0]; others [n0]
template <int MK, class BumpPtr>
__device__ __forceinline__ void med32(const MediumDev &m, const MedF &mf, BumpPtr bumps, float dL0,
                                      f3 P, f3 s, float n_last, float &n, float &nl, f3 &g,
                                      float &dn) {
    static_assert(!kIndexIn64<MK>, "index taken in double by the march");
    nl = 0.0f;
    if constexpr (MK == VRT_MEDIUM_HOMOGENEOUS) {
        n = mf.q[0];
        nl = mf.q[1];
        g = mkf(0, 0, 0);
        dn = 0.0f;
    } else if constexpr (MK == VRT_MEDIUM_LINEAR) {
        g = mkf(mf.q[1], mf.q[2], mf.q[3]);
        const float v = dotf(g, P);
        n = mf.q[0] + v;
        nl = ((mf.q[0] - n) + v) + mf.q[4];
        dn = dotf(g, s);
    } else if constexpr (MK == VRT_MEDIUM_LUNEBURG) {
        // n^2 = 2 - u, u = |P-C|^2/R^2:  n_i - n_{i-1} = -(u_i - u_{i-1}) / (n_i + n_{i-1}),
        // u_i - u_{i-1} = (2 (P-C).s - |s|^2) / R^2
        const f3 o = mkf(P.x - mf.q[1], P.y - mf.q[2], P.z - mf.q[3]);
        const float u = dotf(o, o) * mf.q[4];
        n = fsqrt(2.0f - u);
        const float k = -mf.q[4] * frcp(n);
        g = mkf(k * o.x, k * o.y, k * o.z);
        const float du = (2.0f * dotf(o, s) - dotf(s, s)) * mf.q[4];
        dn = -du * frcp(n + n_last);
    } else if constexpr (MK == VRT_MEDIUM_FIBER) {
        const float x = P.x - mf.q[3], y = P.y - mf.q[4];
        const float r2 = x * x + y * y;
        const float xp = x - s.x, yp = y - s.y;
        const bool core = r2 <= mf.q[7], core_p = xp * xp + yp * yp <= mf.q[7];
        if (core) {
            n = mf.q[0] * fsqrt(1.0f - 2.0f * mf.q[1] * r2 * frcp(mf.q[7]));
            const float k = -mf.q[5] * frcp(n);
            g = mkf(k * x, k * y, 0.0f);
        } else {
            n = mf.q[6];
            g = mkf(0, 0, 0);
        }
        if (core && core_p) {
            // n^2 difference: -(2 Delta n_c^2 / R^2) (2 (x s_x + y s_y) - s_x^2 - s_y^2)
            const float d2 = 2.0f * (x * s.x + y * s.y) - (s.x * s.x + s.y * s.y);
            dn = -mf.q[5] * d2 * frcp(n + n_last);
        } else {
            dn = n - n_last;
        }
    } else if constexpr (MK == VRT_MEDIUM_GAUSSIAN) {
        // E_k(P_{i-1}) = E_k(P_i) exp(dq_k), dq_k = ((P_i - c_k).s - |s|^2/2) / sigma^2,
        // so n_i - n_{i-1} = -sum A_k E_k(P_i) expm1(dq_k), with A_k expm1 as a
        // polynomial in y = sigma^2 dq_k whose coefficients carry A_k.
        float nn = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, acc = 0.f;
        const float hs2 = -0.5f * dotf(s, s);
        const BumpPtr b = bumps;
        const int K = m.K;
        auto bump_loop = [&](auto deg) {
#pragma unroll 4
            for (int k = 0; k < K; ++k) {
                const BumpPtr bk = b + kBumpF * k;
                const float A = bk[0], e2 = bk[1];
                const float ox = P.x - bk[2], oy = P.y - bk[3], oz = P.z - bk[4];
                const float r2 = ox * ox + oy * oy + oz * oz;
                const float E = __builtin_amdgcn_exp2f(r2 * e2);  // exp(-r^2 / (2 sigma^2))
                nn += A * E;
                const float w = E * bk[5];  // A E / sigma^2
                gx -= w * ox;
                gy -= w * oy;
                gz -= w * oz;
                const float y = __builtin_fmaf(ox, s.x, __builtin_fmaf(oy, s.y, __builtin_fmaf(oz, s.z, hs2)));
                float pa;  // A expm1(y / sigma^2)
                if constexpr (decltype(deg)::value == 3)
                    pa = y * (bk[5] + y * (bk[6] + y * bk[7]));
                else
                    pa = y * (bk[5] + y * (bk[6] + y * (bk[7] + y * (bk[8] + y * bk[9]))));
                acc -= E * pa;
            }
        };
        if (dL0 <= mf.q[1])
            bump_loop(std::integral_constant<int, 3>{});
        else
            bump_loop(std::integral_constant<int, 5>{});
        n = mf.q[0] + nn;
        nl = ((mf.q[0] - n) + nn) + mf.q[2];
        g = mkf(gx, gy, gz);
        dn = acc;
    }
}

}  // namespace vrt
