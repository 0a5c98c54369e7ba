// lane32.h -- one lane of the single-precision compensated VRT march: launch
// and entry of a ray, and one decision + move of the march.  Shared by the
// persistent batch kernel (march_fp32c.hip) and the serving kernel
// (serve.hip).
//
// One lane owns one ray at a time.  The march body per step is the method of
// Sec. II: evaluate n, grad n at P_i, normal N = grad n/|grad n| (Eq. (5)),
// then straight (cases (ii)/(iii)), tangential arc (case (iv)), TIR
// (case (v), Eqs. (19)-(20)) or vectorial Snell (Eqs. (9)-(10)), and the
// constant-OPL move P_{i+1} = P_i + Delta R (Eqs. (3)-(4)), cut at the
// enclosing surface where case (i) refracts the ray out or reflects it.
//
// Precision plan:
//   - n and grad n in single precision; the index difference to the previous
//     point is formed from the move vector (media.h), so mu_i - 1 keeps full
//     relative precision.  Media whose index is taken in double (kIndexIn64)
//     are evaluated once per step at the compensated position, and n(P_{i-1})
//     is kept in double, so dn is the difference of two double indices;
//   - Snell is applied as an increment R - I = (mu-1) I + gamma N with
//     gamma = -sgn(c) (mu-1)(mu+1) / (sqrt(D) + mu |c|), the same root as
//     Eq. (10) without its cancellation;
//   - position and direction are Kahan-compensated float pairs (value = h - c);
//   - the step length Delta = dL0 / n is a float pair (Dh + Dl) formed from
//     dL0 and n as float pairs with one Newton correction, and each move adds
//     Delta I to the position with the product's rounding error, the
//     direction's compensation term and Dl folded into the compensation: a
//     float-rounded step length or a move along the rounded direction alone
//     biases every step the same way (dL0 = 5e-4 rounds 2.5e-8 short), and the
//     drift along the path shifts where the discrete TIR of a turning point
//     lands, which moves the reflected direction by ~1e-6 rad;
//   - the discriminant D = mu^2 c^2 - (mu^2 - 1) is evaluated in double;
//   - near grazing incidence, c^2 <= 4 |mu^2 - 1| -- the only region where a
//     refraction/TIR decision can be taken or where gamma is sensitive to the
//     normal -- the normal, c, D and the new direction are recomputed in
//     double from the compensated position (every TIR goes through here);
//   - launch, entry, surface events and the exit plane run in double;
//   - |I| is not renormalized: the Snell increment keeps |R| = |I| in exact
//     arithmetic and its rounding adds ~1e-11 per step to the compensated sum,
//     so a ray's result depends only on its own steps, never on the lane or
//     the moment that runs it.
//
// Scheduling: the grid is sized to the machine, not to the batch.  When a
// lane's ray ends, the wave counts its idle lanes with a ballot, one lane
// claims that many ray indices with a single atomic, and the indices are
// handed out by prefix count.  Every lane leaves once the queue is exhausted
// and its last ray has ended.
#pragma once

#include "dispatch.h"

namespace vrt {

__device__ __forceinline__ void kahan_add(float &h, float &c, float x) {
    const float y = x - c;
    const float t = h + y;
    c = (t - h) - y;
    h = t;
}
__device__ __forceinline__ void split(double v, float &h, float &c) {
    h = (float)v;
    c = (float)((double)h - v);
}
// Step length Delta = (dh + dl) / (nh + nl) as Dh + Dl (the low parts are
// far below the high ones): a quotient from the hardware reciprocal, its
// exact residual dh - q nh (fma), the low parts' first-order terms, and one
// Newton correction.  Relative error ~1e-13.
__device__ __forceinline__ void step_len(float dh, float dl, float nh, float nl, float &Dh,
                                         float &Dl) {
    const float r = __builtin_amdgcn_rcpf(nh);
    const float q = dh * r;
    float e = __builtin_fmaf(-q, nh, dh);
    e = __builtin_fmaf(-q, nl, e + dl);
    const float c = e * r;
    Dh = q + c;
    Dl = (q - Dh) + c;
}
// Step length in double as Dh + Dl.
__device__ __forceinline__ void step_len64(double v, float &Dh, float &Dl) {
    Dh = (float)v;
    Dl = (float)(v - (double)Dh);
}

// Discretized medium: cached records of the 8 corners of the current cell.
struct GridCache {
    int ci, cj, ck;
    float4 v[8];  // node records (n, h_x, h_y, h_z) at corner dx + 2 dy + 4 dz
};

struct Lane {
    float Phx, Phy, Phz, Pcx, Pcy, Pcz;  // position P = Ph - Pc
    float Ihx, Ihy, Ihz, Icx, Icy, Icz;  // direction I = Ih - Ic
    float sx, sy, sz;                    // last move P_i - P_{i-1}
    float nlb;                           // n(P_{i-1}) = nlb + nld (grid: cell base value
    double nld;                          //   + offset inside the cell; media taken in double:
                                         //   the double index split; other media: nld = 0)
    float Delta, Dl;                     // pending move length Delta + Dl
    uint32_t r, steps, ntir, nbtir, flags;
    bool pending;                        // R = I and Delta set by an event: move without deciding
};

// Trilinear blend of the cached records at the fractional position: the
// index offset from the cell's base value v000 in double (weights from the
// double coordinates, node differences exact in float), and the gradient
// (node differences per spacing) in single precision.
__device__ __forceinline__ void grid_blend(const GridCache &gc, double fx, double fy, double fz,
                                           double &delta, float &gx, float &gy, float &gz) {
    const float base = gc.v[0].x;
    double e[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double a = (double)(gc.v[2 * q].x - base);  // exact: nearby float values
        const double b = (double)(gc.v[2 * q + 1].x - base);
        e[q] = a + fx * (b - a);
    }
    const double b0 = e[0] + fy * (e[1] - e[0]), b1 = e[2] + fy * (e[3] - e[2]);
    delta = b0 + fz * (b1 - b0);
    const float ffx = (float)fx, ffy = (float)fy, ffz = (float)fz;
    float gxa[4], gya[4], gza[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 a = gc.v[2 * q], c = gc.v[2 * q + 1];
        gxa[q] = a.y + ffx * (c.y - a.y);
        gya[q] = a.z + ffx * (c.z - a.z);
        gza[q] = a.w + ffx * (c.w - a.w);
    }
    const float gx0 = gxa[0] + ffy * (gxa[1] - gxa[0]), gx1 = gxa[2] + ffy * (gxa[3] - gxa[2]);
    const float gy0 = gya[0] + ffy * (gya[1] - gya[0]), gy1 = gya[2] + ffy * (gya[3] - gya[2]);
    const float gz0 = gza[0] + ffy * (gza[1] - gza[0]), gz1 = gza[2] + ffy * (gza[3] - gza[2]);
    gx = gx0 + ffz * (gx1 - gx0);
    gy = gy0 + ffz * (gy1 - gy0);
    gz = gz0 + ffz * (gz1 - gz0);
}

// Cell and fractional coordinates of P = ph - pc.  Done in double: in float a
// coordinate near 1 carries ~6e-8 of rounding, 1.5e-5 of a 256^3 cell, and
// the trilinear gradient can change by its own size across one cell.
__device__ __forceinline__ void grid_locate(const MediumDev &m, float phx, float phy, float phz,
                                            float pcx, float pcy, float pcz, int &ci, int &cj,
                                            int &ck, double &fx, double &fy, double &fz) {
    const double u = ((double)phx - (double)pcx - m.lo[0]) * m.inv_h[0];
    const double v = ((double)phy - (double)pcy - m.lo[1]) * m.inv_h[1];
    const double w = ((double)phz - (double)pcz - m.lo[2]) * m.inv_h[2];
    ci = min(max((int)floor(u), 0), m.nx - 2);
    cj = min(max((int)floor(v), 0), m.ny - 2);
    ck = min(max((int)floor(w), 0), m.nz - 2);
    fx = u - (double)ci;
    fy = v - (double)cj;
    fz = w - (double)ck;
}

__device__ __forceinline__ void grid_fetch(const MediumDev &m, const float4 *__restrict__ rec, GridCache &gc, int ci, int cj,
                                           int ck) {
    gc.ci = ci;
    gc.cj = cj;
    gc.ck = ck;
    const size_t sx = 1, sy = (size_t)m.nx, sz = (size_t)m.nx * m.ny;
    const size_t o = (size_t)ck * sz + (size_t)cj * sy + ci;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        gc.v[j] = rec[o + (j & 1) * sx + ((j >> 1) & 1) * sy + ((j >> 2) & 1) * sz];
}

// n, grad n and n(P_i) - n(P_{i-1}) for the discretized medium.  The index
// is kept as cell base value + offset (nb, nd): the base is a node value and
// the offset is accurate to double rounding, so the difference to the
// previous point's (nlb, nld) keeps full precision within and across cells.
__device__ __forceinline__ void grid32(const MediumDev &m, const float4 *__restrict__ rec, GridCache &gc, float px, float py, float pz,
                                       float pcx, float pcy, float pcz, float nlb, double nld,
                                       float &n, float &nb, double &nd, float &gx, float &gy,
                                       float &gz, float &dn) {
    int ci, cj, ck;
    double fx, fy, fz;
    grid_locate(m, px, py, pz, pcx, pcy, pcz, ci, cj, ck, fx, fy, fz);
    if (ci != gc.ci || cj != gc.cj || ck != gc.ck) grid_fetch(m, rec, gc, ci, cj, ck);
    double delta;
    grid_blend(gc, fx, fy, fz, delta, gx, gy, gz);
    gx *= m.finv_h[0];  // records hold node differences per node spacing
    gy *= m.finv_h[1];
    gz *= m.finv_h[2];
    nb = gc.v[0].x;
    nd = delta;
    n = (float)((double)nb + nd);
    dn = (float)((double)(nb - nlb) + (nd - nld));  // nb - nlb exact: nearby node values
}

// n and grad n in double at P from the cell records (exact node differences
// per spacing): the cached cell when P lies in it, else the cell is loaded.
__device__ inline void grid_eval64(const MediumDev &m, const float4 *__restrict__ rec, const GridCache &gc, d3 P, double &n,
                                   d3 &g) {
    const int nn[3] = {m.nx, m.ny, m.nz};
    int c[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double x = get(P, a);
        x = x < m.lo[a] ? m.lo[a] : (x > m.hi[a] ? m.hi[a] : x);
        const double u = (x - m.lo[a]) / m.h[a];
        int ci = (int)floor(u);
        ci = ci < 0 ? 0 : (ci > nn[a] - 2 ? nn[a] - 2 : ci);
        c[a] = ci;
        f[a] = u - (double)ci;
    }
    const bool cached = c[0] == gc.ci && c[1] == gc.cj && c[2] == gc.ck;
    const size_t sy = (size_t)m.nx, sz = (size_t)m.nx * m.ny;
    const size_t o = (size_t)c[2] * sz + (size_t)c[1] * sy + c[0];
    n = 0.0;
    g = mk(0, 0, 0);
    for (int j = 0; j < 8; ++j) {
        const float4 r = cached ? gc.v[j]
                                : rec[o + (j & 1) + ((j >> 1) & 1) * sy + ((j >> 2) & 1) * sz];
        const double w = ((j & 1) ? f[0] : 1.0 - f[0]) * ((j & 2) ? f[1] : 1.0 - f[1]) *
                         ((j & 4) ? f[2] : 1.0 - f[2]);
        n += w * (double)r.x;
        g.x += w * (double)r.y;
        g.y += w * (double)r.z;
        g.z += w * (double)r.w;
    }
    g = mk(g.x / m.h[0], g.y / m.h[1], g.z / m.h[2]);
}

template <int MK>
__device__ __forceinline__ void write_out(const RaysDev<float> &io, const Lane &L, d3 P, d3 D,
                                          uint32_t status) {
    const uint32_t r = L.r;
    io.ox[r] = (float)P.x;
    io.oy[r] = (float)P.y;
    io.oz[r] = (float)P.z;
    io.odx[r] = (float)D.x;
    io.ody[r] = (float)D.y;
    io.odz[r] = (float)D.z;
    io.status[r] = status;
    io.steps[r] = L.steps;
    io.n_tir[r] = L.ntir;
    io.n_btir[r] = L.nbtir;
    io.flags[r] = L.flags;
}

// Index at a surface point in the representation the march keeps.
template <int MK>
__device__ __forceinline__ void index_at_event(const MediumDev &m, const float4 *__restrict__ rec, GridCache &gc, d3 P,
                                               float &nlb,
                                               double &nld) {
    if constexpr (MK == VRT_MEDIUM_GRID) {
        float n, gx, gy, gz, dn;
        gc.ci = -1;
        float phx, phy, phz, pcx, pcy, pcz;
        split(P.x, phx, pcx);
        split(P.y, phy, pcy);
        split(P.z, phz, pcz);
        grid32(m, rec, gc, phx, phy, phz, pcx, pcy, pcz, 0.f, 0.0, n, nlb, nld, gx, gy, gz, dn);
    } else if constexpr (kIndexIn64<MK>) {
        const double n = index64<MK>(m, P);
        nlb = (float)n;
        nld = n - (double)nlb;
    } else {
        nlb = (float)index64<MK>(m, P);
        nld = 0.0;
    }
}

// Start ray L.r: launch state, straight flight in the surroundings and entry
// refraction (double).  Returns false if the ray already ended (written).
template <int MK>
__device__ bool lane_init(const MediumDev &m, const float4 *__restrict__ rec, const BoundaryDev &b, const TraceDev &t,
                          const RaysDev<float> &io, Lane &L, GridCache &gc) {
    const uint32_t r = L.r;
    L.steps = L.ntir = L.nbtir = L.flags = 0;
    L.sx = L.sy = L.sz = 0.0f;
    d3 P0 = mk(io.px[r], io.py[r], io.pz[r]);
    d3 d0 = mk(io.dx[r], io.dy[r], io.dz[r]);
    const double l0 = sqrt(dot(d0, d0));
    if (!isfinite(P0.x) || !isfinite(P0.y) || !isfinite(P0.z) || !isfinite(l0) || !(l0 > 0.0)) {
        write_out<MK>(io, L, P0, d0, VRT_RAY_INVALID_INPUT);
        return false;
    }
    const d3 I = mk(d0.x / l0, d0.y / l0, d0.z / l0);
    if (surf_inside_strict(b, P0)) {
        split(P0.x, L.Phx, L.Pcx);
        split(P0.y, L.Phy, L.Pcy);
        split(P0.z, L.Phz, L.Pcz);
        split(I.x, L.Ihx, L.Icx);
        split(I.y, L.Ihy, L.Icy);
        split(I.z, L.Ihz, L.Icz);
        index_at_event<MK>(m, rec, gc, P0, L.nlb, L.nld);
        L.pending = false;
        return true;
    }
    double tt;
    int face;
    if (!surf_entry(b, P0, I, tt, face)) {
        write_out<MK>(io, L, P0, I, VRT_RAY_MISSED);
        return false;
    }
    d3 P = P0 + tt * I;
    surf_snap(b, P, face);
    const d3 N = surf_normal(b, P, face);
    const double n_in = index64<MK>(m, P);
    const double mu = m.n_amb / n_in, c = dot(N, I);
    const double D = 1.0 - mu * mu * (1.0 - c * c);
    if (near_critical(mu, c, D, t.crit_rad)) L.flags |= VRT_FLAG_NEAR_CRITICAL;
    if (D <= 0.0) {
        write_out<MK>(io, L, P, reflect64(I, N, c), VRT_RAY_REFLECTED_AT_ENTRY);
        return false;
    }
    const d3 R = snell64(I, N, mu, c, D);
    split(P.x, L.Phx, L.Pcx);
    split(P.y, L.Phy, L.Pcy);
    split(P.z, L.Phz, L.Pcz);
    split(R.x, L.Ihx, L.Icx);
    split(R.y, L.Ihy, L.Icy);
    split(R.z, L.Ihz, L.Icz);
    index_at_event<MK>(m, rec, gc, P, L.nlb, L.nld);
    step_len64(t.dL0 / n_in, L.Delta, L.Dl);
    L.pending = true;
    return true;
}

// One decision (unless pending) and one move.  Returns false when the ray
// ended (written).
template <int MK, class BumpPtr>
__device__ __forceinline__ bool lane_step(const MediumDev &m, const MedF &mf, BumpPtr bumps,
                                          const float4 *__restrict__ rec, const BoundaryDev &b,
                                          const TraceDev &t, const RaysDev<float> &io, Lane &L,
                                          GridCache &gc, float dL0, float eps_tan, float mrg,
                                          float crit_f) {
    if (!L.pending) {
        const float dL0l = (float)(t.dL0 - (double)dL0);  // dL0 = dL0 + dL0l
        float ni, gx, gy, gz, dn, nb = 0.f, nl = 0.f;
        double nd = 0.0;
        float n_last = L.nlb;  // float-evaluated analytic media keep nld = 0
        if constexpr (MK == VRT_MEDIUM_GRID) n_last = (float)((double)L.nlb + L.nld);
        if constexpr (MK == VRT_MEDIUM_GRID) {
            grid32(m, rec, gc, L.Phx, L.Phy, L.Phz, L.Pcx, L.Pcy, L.Pcz, L.nlb, L.nld, ni, nb, nd, gx,
                   gy, gz, dn);
            nl = (float)(((double)nb + nd) - (double)ni);
        } else if constexpr (kIndexIn64<MK>) {
            // n and grad n in double at the compensated position; n(P_{i-1}) is
            // kept as nlb + nld, so dn is a difference of two double indices
            const d3 P64 = mk((double)L.Phx - L.Pcx, (double)L.Phy - L.Pcy, (double)L.Phz - L.Pcz);
            double n64;
            d3 g64;
            med64<MK>(m, P64, n64, g64);
            ni = nb = (float)n64;
            nd = n64 - (double)nb;
            nl = (float)nd;
            dn = (float)(n64 - ((double)L.nlb + L.nld));
            gx = (float)g64.x;
            gy = (float)g64.y;
            gz = (float)g64.z;
            (void)n_last;
        } else {
            f3 g;
            med32<MK>(m, mf, bumps, dL0, mkf(L.Phx, L.Phy, L.Phz), mkf(L.sx, L.sy, L.sz), n_last,
                      ni, nl, g, dn);
            gx = g.x;
            gy = g.y;
            gz = g.z;
            nb = ni;
        }
        float incx = 0.f, incy = 0.f, incz = 0.f, Delta, Dl;
        const float gl2 = gx * gx + gy * gy + gz * gz;
        if (!(gl2 > 0.0f) || !isfinite(gl2)) {  // cases (ii)/(iii): straight
            step_len(dL0, dL0l, ni, nl, Delta, Dl);
            L.flags |= VRT_FLAG_STRAIGHT;
        } else {
            const float inv = rsqrtf(gl2);
            const float Nx = gx * inv, Ny = gy * inv, Nz = gz * inv;  // Eq. (5)
            const float c = (Nx * L.Ihx + Ny * L.Ihy + Nz * L.Ihz) -
                            (Nx * L.Icx + Ny * L.Icy + Nz * L.Icz);
            if (fabsf(c) <= eps_tan) {
                // case (iv): arc with curvature grad n / n, Eqs. (16)-(18);
                // dn along the probe Delta N in difference form
                step_len(dL0, dL0l, ni, nl, Delta, Dl);
                const float qx = Delta * Nx, qy = Delta * Ny, qz = Delta * Nz;
                float np, dnp;
                if constexpr (MK == VRT_MEDIUM_GRID) {
                    float pb, px, py, pz;
                    double pd;
                    GridCache g2 = gc;
                    grid32(m, rec, g2, L.Phx + qx, L.Phy + qy, L.Phz + qz, L.Pcx, L.Pcy, L.Pcz, nb, nd, np,
                           pb, pd, px, py, pz, dnp);
                } else if constexpr (kIndexIn64<MK>) {
                    const d3 Q64 = mk((double)L.Phx - L.Pcx + qx, (double)L.Phy - L.Pcy + qy,
                                      (double)L.Phz - L.Pcz + qz);
                    double nq;
                    d3 gq;
                    med64<MK>(m, Q64, nq, gq);
                    np = (float)nq;
                    dnp = (float)(nq - ((double)nb + nd));
                } else {
                    f3 gp;
                    float npl;
                    med32<MK>(m, mf, bumps, dL0, mkf(L.Phx + qx, L.Phy + qy, L.Phz + qz), mkf(qx, qy, qz), ni,
                              np, npl, gp, dnp);
                }
                const float a = dnp * frcp(2.0f * ni);
                const float w = fsqrt(fmaxf(0.0f, 1.0f - a * a));
                const float k = -a * a / (1.0f + w);  // sqrt(1-a^2) - 1 without cancellation
                incx = k * L.Ihx + a * Nx;
                incy = k * L.Ihy + a * Ny;
                incz = k * L.Ihz + a * Nz;
                L.flags |= VRT_FLAG_TANGENT;
            } else {
                const float m1 = -dn * frcp(ni);  // mu_i - 1, mu_i = n_{i-1} / n_i
                if (c * c <= 4.0f * fabsf(m1) * (2.0f + m1)) {
                    // near grazing: the step is taken in double -- n at P_i and
                    // P_{i-1}, the normal, c, D and R (Eqs. (5), (9)-(10), (19)-(20))
                    const d3 P64 = mk((double)L.Phx - L.Pcx, (double)L.Phy - L.Pcy,
                                      (double)L.Phz - L.Pcz);
                    const d3 Pp64 = P64 - mk((double)L.sx, (double)L.sy, (double)L.sz);
                    const d3 I64 = mk((double)L.Ihx - L.Icx, (double)L.Ihy - L.Icy,
                                      (double)L.Ihz - L.Icz);
                    d3 g64, gp;
                    double ni64, np64;
                    if constexpr (MK == VRT_MEDIUM_GRID) {
                        grid_eval64(m, rec, gc, P64, ni64, g64);
                        grid_eval64(m, rec, gc, Pp64, np64, gp);
                    } else {
                        med64<MK>(m, P64, ni64, g64);
                        med64<MK>(m, Pp64, np64, gp);
                    }
                    const double gl = sqrt(dot(g64, g64));
                    const d3 N = mk(g64.x / gl, g64.y / gl, g64.z / gl);
                    const double cd = dot(N, I64);
                    const double mu = np64 / ni64;
                    const double D = 1.0 - mu * mu * (1.0 - cd * cd);
                    if (near_critical(mu, cd, D, t.crit_rad)) L.flags |= VRT_FLAG_NEAR_CRITICAL;
                    if (mu < 1.0 && fabs(cd) < t.crit_rad) L.flags |= VRT_FLAG_NEAR_GRAZING;
                    d3 R;
                    if (D <= 0.0) {  // case (v): reflect, Delta_{i-1} (Eq. (20))
                        R = reflect64(I64, N, cd);
                        step_len64(t.dL0 / np64, Delta, Dl);
                        L.ntir++;
                    } else {
                        R = snell64(I64, N, mu, cd, D);
                        step_len64(t.dL0 / ni64, Delta, Dl);
                    }
                    split(R.x, L.Ihx, L.Icx);
                    split(R.y, L.Ihy, L.Icy);
                    split(R.z, L.Ihz, L.Icz);
                } else {  // Eqs. (9)-(10) as an increment
                    // D = mu^2 c^2 - (mu^2 - 1) >= (3/4) mu^2 c^2 here: no cancellation,
                    // float keeps it to a few ulp.  The near-critical window needs
                    // |D| < 2 mu^2 crit_rad (the bound in near_critical); screen for
                    // it with 1 % slack and decide it in double.
                    const float muf = 1.0f + m1;
                    const float D = muf * muf * c * c - m1 * (2.0f + m1);
                    if (m1 > 0.0f && D < 2.02f * muf * muf * crit_f) {
                        const double mu = 1.0 + (double)m1, cd = (double)c;
                        const double Dd = mu * mu * cd * cd - (double)m1 * (2.0 + (double)m1);
                        if (near_critical(mu, cd, Dd, t.crit_rad)) L.flags |= VRT_FLAG_NEAR_CRITICAL;
                    }
                    const float sD = fsqrt(D);
                    const float q = m1 * (2.0f + m1) * frcp(sD + muf * fabsf(c));
                    const float gam = c > 0.0f ? -q : q;  // -sgn(c) q, q signed
                    incx = m1 * L.Ihx + gam * Nx;
                    incy = m1 * L.Ihy + gam * Ny;
                    incz = m1 * L.Ihz + gam * Nz;
                    step_len(dL0, dL0l, ni, nl, Delta, Dl);
                }
            }
        }
        L.nlb = nb;
        if constexpr (MK == VRT_MEDIUM_GRID || kIndexIn64<MK>) L.nld = nd;
        kahan_add(L.Ihx, L.Icx, incx);
        kahan_add(L.Ihy, L.Icy, incy);
        kahan_add(L.Ihz, L.Icz, incz);
        L.Delta = Delta;
        L.Dl = Dl;
    }
    L.pending = false;
    // ---- move (Eqs. (3)-(4)), cut at the enclosing surface (case (i)) ----
    const float Delta = L.Delta, Dl = L.Dl;
    const float mvx = Delta * L.Ihx, mvy = Delta * L.Ihy, mvz = Delta * L.Ihz;
    bool full = surf_inside_margin(b, L.Phx + mvx, L.Phy + mvy, L.Phz + mvz, mrg);
    d3 P64, R64;
    double tx = 0.0;
    int face = 0;
    if (!full) {  // near or at the surface: decide in double
        P64 = mk((double)L.Phx - L.Pcx, (double)L.Phy - L.Pcy, (double)L.Phz - L.Pcz);
        R64 = mk((double)L.Ihx - L.Icx, (double)L.Ihy - L.Icy, (double)L.Ihz - L.Icz);
        tx = surf_exit(b, P64, R64, face);
        const double D64 = (double)Delta + (double)Dl;
        full = tx > D64;
        if (tx < 3.0 * D64) {  // distance of the step end from the surface
            const d3 Ne = surf_normal(b, P64 + tx * R64, face);
            if (fabs(tx - D64) * fabs(dot(R64, Ne)) < t.tie_eps)
                L.flags |= VRT_FLAG_NEAR_TIE;
        }
    }
    L.steps++;
    if (full) {
        // P += (Delta + Dl)(Ih - Ic): the float move, then its rounding error,
        // Dl and the direction's compensation into the compensation term
        const float ex = __builtin_fmaf(Delta, L.Ihx, -mvx) + (Dl * L.Ihx - Delta * L.Icx);
        const float ey = __builtin_fmaf(Delta, L.Ihy, -mvy) + (Dl * L.Ihy - Delta * L.Icy);
        const float ez = __builtin_fmaf(Delta, L.Ihz, -mvz) + (Dl * L.Ihz - Delta * L.Icz);
        kahan_add(L.Phx, L.Pcx, mvx);
        kahan_add(L.Phy, L.Pcy, mvy);
        kahan_add(L.Phz, L.Pcz, mvz);
        L.Pcx -= ex;
        L.Pcy -= ey;
        L.Pcz -= ez;
        L.sx = mvx;
        L.sy = mvy;
        L.sz = mvz;
        if ((int64_t)L.steps >= t.max_steps) {
            write_out<MK>(io, L,
                          mk((double)L.Phx - L.Pcx, (double)L.Phy - L.Pcy, (double)L.Phz - L.Pcz),
                          mk((double)L.Ihx - L.Icx, (double)L.Ihy - L.Icy, (double)L.Ihz - L.Icz),
                          VRT_RAY_TRUNCATED);
            return false;
        }
        return true;
    }
    // surface event in double
    d3 P = P64 + tx * R64;
    surf_snap(b, P, face);
    const d3 N = surf_normal(b, P, face);
    const double n_last = (double)L.nlb + L.nld;
    const double mu = n_last / m.n_amb, c = dot(N, R64);
    const double D = 1.0 - mu * mu * (1.0 - c * c);
    if (near_critical(mu, c, D, t.crit_rad)) L.flags |= VRT_FLAG_NEAR_CRITICAL;
    if (D <= 0.0) {  // reflected back inside
        const d3 R = reflect64(R64, N, c);
        split(P.x, L.Phx, L.Pcx);
        split(P.y, L.Phy, L.Pcy);
        split(P.z, L.Phz, L.Pcz);
        split(R.x, L.Ihx, L.Icx);
        split(R.y, L.Ihy, L.Icy);
        split(R.z, L.Ihz, L.Icz);
        step_len64(t.dL0 / n_last, L.Delta, L.Dl);
        index_at_event<MK>(m, rec, gc, P, L.nlb, L.nld);
        L.nbtir++;
        L.flags |= VRT_FLAG_BOUNDARY_TIR;
        L.pending = true;
        if ((int64_t)L.steps >= t.max_steps) {
            write_out<MK>(io, L, P, R, VRT_RAY_TRUNCATED);
            return false;
        }
        return true;
    }
    const d3 Ro = snell64(R64, N, mu, c, D);
    uint32_t st = VRT_RAY_EXITED;
    d3 Po = P;
    if (t.has_plane) {
        if (!(Ro.z > 0.0) || (t.plane_z - P.z) / Ro.z < 0.0) {
            st = VRT_RAY_NO_PLANE;
        } else {
            const double s = (t.plane_z - P.z) / Ro.z;
            Po = mk(P.x + s * Ro.x, P.y + s * Ro.y, t.plane_z);
        }
    }
    write_out<MK>(io, L, Po, Ro, st);
    return false;
}

}  // namespace vrt
