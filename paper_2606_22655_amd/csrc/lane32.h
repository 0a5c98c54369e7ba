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
// The tangential rule's new direction R = (w I + a N) / |w I + a N|,
// w = sqrt(1 - a^2), Eqs. (16)-(18), as the increment R - I.  With
// c = N.I (|c| <= eps_tan), |w I + a N|^2 = 1 + 2 a w c = L^2, and
// R - I = (k I + a N) / L with k = w - L = -(a^2 + 2 a w c) / (w + L), formed
// without cancellation; at c = 0, L = 1 and k = -a^2 / (1 + w).
__device__ __forceinline__ void tangent_increment(float a, float c, float Ix, float Iy, float Iz,
                                                  float Nx, float Ny, float Nz, float &incx,
                                                  float &incy, float &incz) {
    const float w = fsqrt(fmaxf(0.0f, 1.0f - a * a));
    const float x = 2.0f * a * w * c;
    const float L = fsqrt(1.0f + x);
    const float k = -(a * a + x) / (w + L);
    const float il = frcp(L);
    incx = (k * Ix + a * Nx) * il;
    incy = (k * Iy + a * Ny) * il;
    incz = (k * Iz + a * Nz) * il;
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

// Discretized medium: the current cell, its origin and its 8 corner records.
struct GridCache {
    int ci, cj, ck;             // cell indices; ci < 0: none (locate in double)
    float ox, oy, oz;           // cell origin lo + c h as float pairs: head ...
    float olx, oly, olz;        //   ... and low part
    float4 v[8];  // node records (n, h_x, h_y, h_z) at corner dx + 2 dy + 4 dz
};

// Forget the cached cell (the position jumped: entry, surface event).
__device__ __forceinline__ void grid_invalidate(GridCache &gc) {
    gc.ci = -1;
    gc.ox = gc.oy = gc.oz = __builtin_nanf("");
}

struct Lane {
    float Phx, Phy, Phz, Pcx, Pcy, Pcz;  // position P = Ph - Pc
    float Ihx, Ihy, Ihz, Icx, Icy, Icz;  // direction I = Ih - Ic
    float sx, sy, sz;                    // last move P_i - P_{i-1}
    float nlb;                           // n(P_{i-1}) = nlb + nld (media taken in double:
    double nld;                          //   the double index split; other media: nld = 0)
    float nlo;                           // grid: n(P_{i-1}) = nlb + nlo (base node value +
                                         //   offset inside the cell)
    float Delta, Dl;                     // pending move length Delta + Dl
    uint32_t r, steps, ntir, nbtir, flags;
    bool pending;                        // R = I and Delta set by an event: move without deciding
};

// Load cell (ci, cj, ck): its origin (double, kept as a float pair) and the
// records of its 8 corners.
__device__ __forceinline__ void grid_fetch(const MediumDev &m, const float4 *__restrict__ rec,
                                           GridCache &gc, int ci, int cj, int ck) {
    gc.ci = ci;
    gc.cj = cj;
    gc.ck = ck;
    const double ox = m.lo[0] + (double)ci * m.h[0], oy = m.lo[1] + (double)cj * m.h[1],
                 oz = m.lo[2] + (double)ck * m.h[2];
    gc.ox = (float)ox;
    gc.oy = (float)oy;
    gc.oz = (float)oz;
    gc.olx = (float)(ox - (double)gc.ox);
    gc.oly = (float)(oy - (double)gc.oy);
    gc.olz = (float)(oz - (double)gc.oz);
    const size_t sx = 1, sy = (size_t)m.nx, sz = (size_t)m.nx * m.ny;
    const size_t o = (size_t)ck * sz + (size_t)cj * sy + ci;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        gc.v[j] = rec[o + (j & 1) * sx + ((j >> 1) & 1) * sy + ((j >> 2) & 1) * sz];
}

// Fractional coordinate of P = ph - pc along one axis of the cell whose
// origin is o + ol: ph - o is exact or rounds at the cell's scale (the two lie
// within about a cell of each other), and the low parts are folded in at that
// scale, so f carries ~1e-7 of a cell -- without a double in the common step.
__device__ __forceinline__ float cell_frac(float ph, float pc, float o, float ol, float inv_h) {
    return (((ph - o) - ol) - pc) * inv_h;
}

// Cell of P and the fractional coordinates in it.  A step moves P by much
// less than a cell, so when P leaves the cached cell the cell index shifts by
// floor(f) along each axis; after an event (no cell cached: the origin is
// NaN, so every f fails the test) P is located in double.  Indices are
// clamped to the grid, where P itself is clamped (a point on the upper faces
// has f = 1 in the last cell).
__device__ __forceinline__ void grid_cell(const MediumDev &m, const float4 *__restrict__ rec,
                                          GridCache &gc, const Lane &L, float &fx, float &fy,
                                          float &fz) {
    fx = cell_frac(L.Phx, L.Pcx, gc.ox, gc.olx, m.finv_h[0]);
    fy = cell_frac(L.Phy, L.Pcy, gc.oy, gc.oly, m.finv_h[1]);
    fz = cell_frac(L.Phz, L.Pcz, gc.oz, gc.olz, m.finv_h[2]);
    if (fx >= 0.0f && fx < 1.0f && fy >= 0.0f && fy < 1.0f && fz >= 0.0f && fz < 1.0f) return;
    int ci, cj, ck;
    if (gc.ci < 0) {
        ci = (int)floor(((double)L.Phx - (double)L.Pcx - m.lo[0]) * m.inv_h[0]);
        cj = (int)floor(((double)L.Phy - (double)L.Pcy - m.lo[1]) * m.inv_h[1]);
        ck = (int)floor(((double)L.Phz - (double)L.Pcz - m.lo[2]) * m.inv_h[2]);
    } else {
        ci = gc.ci + (int)floorf(fx);
        cj = gc.cj + (int)floorf(fy);
        ck = gc.ck + (int)floorf(fz);
    }
    ci = min(max(ci, 0), m.nx - 2);
    cj = min(max(cj, 0), m.ny - 2);
    ck = min(max(ck, 0), m.nz - 2);
    if (ci != gc.ci || cj != gc.cj || ck != gc.ck) {
        grid_fetch(m, rec, gc, ci, cj, ck);
        fx = cell_frac(L.Phx, L.Pcx, gc.ox, gc.olx, m.finv_h[0]);
        fy = cell_frac(L.Phy, L.Pcy, gc.oy, gc.oly, m.finv_h[1]);
        fz = cell_frac(L.Phz, L.Pcz, gc.oz, gc.olz, m.finv_h[2]);
    }
    // P clamped to the grid (the tangential rule's probe may step outside)
    fx = fminf(fmaxf(fx, 0.0f), 1.0f);
    fy = fminf(fmaxf(fy, 0.0f), 1.0f);
    fz = fminf(fmaxf(fz, 0.0f), 1.0f);
}

// Trilinear blend of the cached records at (fx, fy, fz): the index as an
// offset from the cell's first node value (the node differences are exact in
// float for nearby values), and the gradient's node differences per spacing.
__device__ __forceinline__ void grid_blend(const GridCache &gc, float fx, float fy, float fz,
                                           float &delta, float &gx, float &gy, float &gz) {
    const float base = gc.v[0].x;
    float e[4], gxa[4], gya[4], gza[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 a = gc.v[2 * q], c = gc.v[2 * q + 1];
        const float da = a.x - base, dc = c.x - base;
        e[q] = da + fx * (dc - da);
        gxa[q] = a.y + fx * (c.y - a.y);
        gya[q] = a.z + fx * (c.z - a.z);
        gza[q] = a.w + fx * (c.w - a.w);
    }
    const float b0 = e[0] + fy * (e[1] - e[0]), b1 = e[2] + fy * (e[3] - e[2]);
    delta = b0 + fz * (b1 - b0);
    const float gx0 = gxa[0] + fy * (gxa[1] - gxa[0]), gx1 = gxa[2] + fy * (gxa[3] - gxa[2]);
    const float gy0 = gya[0] + fy * (gya[1] - gya[0]), gy1 = gya[2] + fy * (gya[3] - gya[2]);
    const float gz0 = gza[0] + fy * (gza[1] - gza[0]), gz1 = gza[2] + fy * (gza[3] - gza[2]);
    gx = gx0 + fz * (gx1 - gx0);
    gy = gy0 + fz * (gy1 - gy0);
    gz = gz0 + fz * (gz1 - gz0);
}

// n at P in double from the node values (trilinear, P clamped to the grid):
// the index at surface events and at the tangential rule's probe.
__device__ inline double grid_index64(const MediumDev &m, d3 P) {
    int c[3];
    double f[3];
    grid_cell64(m, P, c, f);
    const size_t sy = (size_t)m.nx, sz = (size_t)m.nx * m.ny;
    const size_t o = (size_t)c[2] * sz + (size_t)c[1] * sy + c[0];
    double n = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                                 (dz ? f[2] : 1.0 - f[2]);
                n += w * (double)m.grid[o + dx + dy * sy + dz * sz];
            }
    return n;
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
__device__ __forceinline__ void index_at_event(const MediumDev &m, GridCache &gc, d3 P, Lane &L) {
    if constexpr (MK == VRT_MEDIUM_GRID) {
        grid_invalidate(gc);
        const double n = grid_index64(m, P);
        L.nlb = (float)n;
        L.nlo = (float)(n - (double)L.nlb);
    } else if constexpr (kIndexIn64<MK>) {
        const double n = index64<MK>(m, P);
        L.nlb = (float)n;
        L.nld = n - (double)L.nlb;
    } else {
        L.nlb = (float)index64<MK>(m, P);
        L.nld = 0.0;
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
        index_at_event<MK>(m, gc, P0, L);
        L.Delta = L.Dl = 0.0f;  // set by the first decision (the grid's request reads it)
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
    index_at_event<MK>(m, gc, P, L);
    step_len64(t.dL0 / n_in, L.Delta, L.Dl);
    L.pending = true;
    return true;
}

// The state of a ray after its launch and entry (lane_init), as the entry
// kernel leaves it for a march kernel that starts rays from it (lane_load):
// the march kernel then holds no double-precision entry code, which for the
// grid medium is where its registers peak.  80 bytes.
struct alignas(16) EntryState {
    float Phx, Phy, Phz, Pcx, Pcy, Pcz;
    float Ihx, Ihy, Ihz, Icx, Icy, Icz;
    float nlb, nlo;
    double nld;
    float Delta, Dl;
    uint32_t flags;
    uint32_t state;  // kEntered, kInside, or kEnded (outputs already written)
};
static_assert(sizeof(EntryState) == 80, "entry state layout");
constexpr uint32_t kEntered = 0, kInside = 1, kEnded = 2;

template <int MK>
__device__ __forceinline__ void entry_store(const Lane &L, bool active, EntryState &e) {
    if (!active) {
        e = EntryState{};
        e.state = kEnded;
        return;
    }
    e.Phx = L.Phx; e.Phy = L.Phy; e.Phz = L.Phz;
    e.Pcx = L.Pcx; e.Pcy = L.Pcy; e.Pcz = L.Pcz;
    e.Ihx = L.Ihx; e.Ihy = L.Ihy; e.Ihz = L.Ihz;
    e.Icx = L.Icx; e.Icy = L.Icy; e.Icz = L.Icz;
    e.nlb = L.nlb;
    e.nlo = MK == VRT_MEDIUM_GRID ? L.nlo : 0.0f;
    e.nld = MK == VRT_MEDIUM_GRID ? 0.0 : L.nld;
    e.Delta = L.Delta;
    e.Dl = L.Dl;
    e.flags = L.flags;
    e.state = L.pending ? kEntered : kInside;
}

// Start ray L.r from its stored entry state.  Returns false if the ray ended
// at its launch or entry (its outputs are written already).
template <int MK>
__device__ __forceinline__ bool lane_load(const EntryState *__restrict__ es, Lane &L,
                                          GridCache &gc) {
    const EntryState &e = es[L.r];
    if (e.state == kEnded) return false;
    L.steps = L.ntir = L.nbtir = 0;
    L.flags = e.flags;
    L.sx = L.sy = L.sz = 0.0f;
    L.Phx = e.Phx; L.Phy = e.Phy; L.Phz = e.Phz;
    L.Pcx = e.Pcx; L.Pcy = e.Pcy; L.Pcz = e.Pcz;
    L.Ihx = e.Ihx; L.Ihy = e.Ihy; L.Ihz = e.Ihz;
    L.Icx = e.Icx; L.Icy = e.Icy; L.Icz = e.Icz;
    L.nlb = e.nlb;
    if constexpr (MK == VRT_MEDIUM_GRID) L.nlo = e.nlo;
    else L.nld = e.nld;
    L.Delta = e.Delta;
    L.Dl = e.Dl;
    L.pending = e.state == kEntered;
    grid_invalidate(gc);
    return true;
}

// The decision of one step in a discretized medium, in single precision:
// the cell and fractions relative to the cached cell's origin, the trilinear
// blend of its records, the index difference (n_i - n_{i-1} as the difference
// of two base node values, exact, plus that of two in-cell offsets), and the
// discriminant D = mu^2 c^2 - (mu^2 - 1) in float.  Near the critical angle D
// is the difference of two terms of size 2 |mu - 1| ~ 1e-3 that float holds to
// ~1e-10, which places the decision D <= 0 to ~1e-8 rad, far inside the
// 1e-6 rad window where rays are flagged.  Refraction is the increment of
// Eqs. (9)-(10) as for the other media; TIR reflects by -2 c N (Eq. (20)) and
// moves on with Delta_{i-1} = dL0 / n_{i-1}.  The tangential rule probes n in
// double from the node values.  Sets the direction increment, L.Delta, L.Dl
// and the index of P_i as the next step's n(P_{i-1}).
__device__ __forceinline__ void grid_decide(const MediumDev &m, const float4 *__restrict__ rec,
                                            const TraceDev &t, Lane &L, GridCache &gc, float dL0,
                                            float eps_tan, float crit_f, float &incx, float &incy,
                                            float &incz) {
    const float dL0l = (float)(t.dL0 - (double)dL0);  // dL0 = dL0 + dL0l
    float fx, fy, fz, delta, gx, gy, gz;
    grid_cell(m, rec, gc, L, fx, fy, fz);
    grid_blend(gc, fx, fy, fz, delta, gx, gy, gz);
    gx *= m.finv_h[0];  // records hold node differences per node spacing
    gy *= m.finv_h[1];
    gz *= m.finv_h[2];
    const float nb = gc.v[0].x;
    const float ni = nb + delta, nl = (nb - ni) + delta;  // n(P_i) = ni + nl
    const float dn = (nb - L.nlb) + (delta - L.nlo);      // nb - nlb exact: nearby node values
    incx = incy = incz = 0.0f;
    const float gl2 = gx * gx + gy * gy + gz * gz;
    if (!(gl2 > 0.0f) || !isfinite(gl2)) {  // cases (ii)/(iii): straight
        step_len(dL0, dL0l, ni, nl, L.Delta, L.Dl);
        L.flags |= VRT_FLAG_STRAIGHT;
    } else {
        const float inv = rsqrtf(gl2);
        const float Nx = gx * inv, Ny = gy * inv, Nz = gz * inv;  // Eq. (5)
        const float c = (Nx * L.Ihx + Ny * L.Ihy + Nz * L.Ihz) -
                        (Nx * L.Icx + Ny * L.Icy + Nz * L.Icz);
        if (fabsf(c) <= eps_tan) {
            // case (iv): arc with curvature grad n / n, Eqs. (16)-(18); n at the
            // probe P + Delta N in double
            step_len(dL0, dL0l, ni, nl, L.Delta, L.Dl);
            const double D64 = (double)L.Delta + (double)L.Dl;
            const d3 Q = mk((double)L.Phx - L.Pcx + D64 * Nx, (double)L.Phy - L.Pcy + D64 * Ny,
                            (double)L.Phz - L.Pcz + D64 * Nz);
            const float dnp = (float)(grid_index64(m, Q) - ((double)nb + (double)delta));
            tangent_increment(dnp * frcp(2.0f * ni), c, L.Ihx, L.Ihy, L.Ihz, Nx, Ny, Nz, incx, incy,
                              incz);
            L.flags |= VRT_FLAG_TANGENT;
        } else {
            const float m1 = -dn * frcp(ni);  // mu_i - 1, mu_i = n_{i-1} / n_i
            const float muf = 1.0f + m1;
            const float D = muf * muf * c * c - m1 * (2.0f + m1);
            if (m1 > 0.0f && fabsf(D) < 2.02f * muf * muf * crit_f) {
                const double mu = 1.0 + (double)m1, cd = (double)c;
                const double Dd = mu * mu * cd * cd - (double)m1 * (2.0 + (double)m1);
                if (near_critical(mu, cd, Dd, t.crit_rad)) L.flags |= VRT_FLAG_NEAR_CRITICAL;
            }
            if (m1 < 0.0f && fabsf(c) < crit_f) L.flags |= VRT_FLAG_NEAR_GRAZING;
            if (D <= 0.0f) {  // case (v): reflect, move on with Delta_{i-1} (Eq. (20))
                const float c2 = -2.0f * c;
                incx = c2 * Nx;
                incy = c2 * Ny;
                incz = c2 * Nz;
                const float nph = L.nlb + L.nlo, npl = (L.nlb - nph) + L.nlo;
                step_len(dL0, dL0l, nph, npl, L.Delta, L.Dl);
                L.ntir++;
            } else {  // Eqs. (9)-(10) as an increment
                const float sD = fsqrt(D);
                const float q = m1 * (2.0f + m1) * frcp(sD + muf * fabsf(c));
                const float gam = c > 0.0f ? -q : q;  // -sgn(c) q, q signed
                incx = m1 * L.Ihx + gam * Nx;
                incy = m1 * L.Ihy + gam * Ny;
                incz = m1 * L.Ihz + gam * Nz;
                step_len(dL0, dL0l, ni, nl, L.Delta, L.Dl);
            }
        }
    }
    L.nlb = nb;
    L.nlo = delta;
}

// One decision (unless pending) and one move.  Returns false when the ray
// ended (written).
template <int MK, class BumpPtr>
__device__ __forceinline__ bool lane_step(const MediumDev &m, const MedF &mf, BumpPtr bumps,
                                          const float4 *__restrict__ rec, const BoundaryDev &b,
                                          const TraceDev &t, const RaysDev<float> &io, Lane &L,
                                          GridCache &gc, float dL0, float eps_tan, float mrg,
                                          float crit_f) {
    if constexpr (MK == VRT_MEDIUM_GRID) {
        if (!L.pending) {
            float incx, incy, incz;
            grid_decide(m, rec, t, L, gc, dL0, eps_tan, crit_f, incx, incy, incz);
            kahan_add(L.Ihx, L.Icx, incx);
            kahan_add(L.Ihy, L.Icy, incy);
            kahan_add(L.Ihz, L.Icz, incz);
        }
    } else if (!L.pending) {
        const float dL0l = (float)(t.dL0 - (double)dL0);  // dL0 = dL0 + dL0l
        float ni, gx, gy, gz, dn, nb = 0.f, nl = 0.f;
        double nd = 0.0;
        const float n_last = L.nlb;  // float-evaluated analytic media keep nld = 0
        double n64 = 0.0;  // media taken in double: n and grad n at P_i
        d3 g64 = mk(0.0, 0.0, 0.0);
        if constexpr (kIndexIn64<MK>) {
            // n and grad n in double at the compensated position; n(P_{i-1}) is
            // kept as nlb + nld, so dn is a difference of two double indices
            const d3 P64 = mk((double)L.Phx - L.Pcx, (double)L.Phy - L.Pcy, (double)L.Phz - L.Pcz);
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
                if constexpr (kIndexIn64<MK>) {
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
                tangent_increment(dnp * frcp(2.0f * ni), c, L.Ihx, L.Ihy, L.Ihz, Nx, Ny, Nz, incx,
                                  incy, incz);
                L.flags |= VRT_FLAG_TANGENT;
            } else {
                const float m1 = -dn * frcp(ni);  // mu_i - 1, mu_i = n_{i-1} / n_i
                if (c * c <= 4.0f * fabsf(m1) * (2.0f + m1)) {
                    // near grazing: the step is taken in double -- n and the
                    // normal at P_i, c, D and R (Eqs. (5), (9)-(10), (19)-(20)).
                    // Media taken in double have n and grad n at P_i in double
                    // already and evaluate n(P_{i-1}) again at P_i - s; media
                    // evaluated in float take mu = 1 + (mu - 1) from the step's
                    // index difference (its error, ~1e-11, moves the critical
                    // angle by ~1e-9 rad).
                    const d3 I64 = mk((double)L.Ihx - L.Icx, (double)L.Ihy - L.Icy,
                                      (double)L.Ihz - L.Icz);
                    double ni64, mu, np64;
                    d3 gi64;
                    if constexpr (kIndexIn64<MK>) {
                        const d3 Pp64 = mk((double)L.Phx - L.Pcx - (double)L.sx,
                                           (double)L.Phy - L.Pcy - (double)L.sy,
                                           (double)L.Phz - L.Pcz - (double)L.sz);
                        d3 gp;
                        med64<MK>(m, Pp64, np64, gp);
                        ni64 = n64;
                        gi64 = g64;
                        mu = np64 / ni64;
                    } else {
                        const d3 P64 = mk((double)L.Phx - L.Pcx, (double)L.Phy - L.Pcy,
                                          (double)L.Phz - L.Pcz);
                        med64<MK>(m, P64, ni64, gi64);
                        mu = 1.0 + (double)m1;
                        np64 = mu * ni64;
                    }
                    const double gl = sqrt(dot(gi64, gi64));
                    const d3 N = mk(gi64.x / gl, gi64.y / gl, gi64.z / gl);
                    const double cd = dot(N, I64);
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
        if constexpr (kIndexIn64<MK>) L.nld = nd;
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
    const double n_last =
        (double)L.nlb + (MK == VRT_MEDIUM_GRID ? (double)L.nlo : L.nld);  // n(P_{i-1})
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
        index_at_event<MK>(m, gc, P, L);
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
