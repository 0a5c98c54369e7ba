// lane64.h -- one ray of the plain double-precision VRT march (Sec. II),
// shared by the batch kernel (march_fp64.hip) and the N2P design sweep
// (design.hip).  Include it after `#pragma clang fp contract(off)` so that
// every operation is correctly rounded as written.
#pragma once

#include "dispatch.h"
#include "media.h"

namespace vrt {

struct Out64 {
    d3 P, D;
    uint32_t status, steps, ntir, nbtir, flags;
};

// Polyline recorders: NoPath records nothing (the batch kernels); PathRec
// stores the points of the polyline -- the launch point, the entry point,
// every step's end and every point where a step meets the surface -- at
// buf + k * stride for point k < cap, and counts them all.
struct NoPath {
    __device__ __forceinline__ void add(const d3 &) {}
};
struct PathRec {
    double *buf;
    uint64_t cap, n;
    size_t stride;
    __device__ __forceinline__ void add(const d3 &P) {
        if (n < cap) {
            double *q = buf + n * stride;
            q[0] = P.x;
            q[1] = P.y;
            q[2] = P.z;
        }
        ++n;
    }
};

template <int MK, class Path>
__device__ void trace_ray64(const MediumDev &m, const BoundaryDev &b, const TraceDev &t, d3 P0,
                            d3 d0, Out64 &o, Path &path) {
    o.P = P0;
    o.D = d0;
    o.status = VRT_RAY_EXITED;
    o.steps = o.ntir = o.nbtir = o.flags = 0;
    const double l0 = sqrt(dot(d0, d0));
    if (!isfinite(P0.x) || !isfinite(P0.y) || !isfinite(P0.z) || !isfinite(l0) || !(l0 > 0.0)) {
        o.status = VRT_RAY_INVALID_INPUT;
        return;
    }
    d3 I = mk(d0.x / l0, d0.y / l0, d0.z / l0);  // unit launch direction
    d3 P = P0, R = I;
    path.add(P);
    double n_last, Delta = 0.0;  // n_last = n at the previous polyline point
    bool decide;
    if (surf_inside_strict(b, P)) {
        n_last = index64<MK>(m, P);
        decide = true;
    } else {
        double tt;
        int face;
        if (!surf_entry(b, P, I, tt, face)) {
            o.status = VRT_RAY_MISSED;
            o.D = I;
            return;
        }
        P = P + tt * I;  // straight in the surroundings (case (iii))
        surf_snap(b, P, face);
        path.add(P);
        d3 N = surf_normal(b, P, face);
        double n_in = index64<MK>(m, P);
        double mu = m.n_amb / n_in, c = dot(N, I);
        double D = 1.0 - mu * mu * (1.0 - c * c);
        if (near_critical(mu, c, D, t.crit_rad)) o.flags |= VRT_FLAG_NEAR_CRITICAL;
        if (D <= 0.0) {
            o.status = VRT_RAY_REFLECTED_AT_ENTRY;
            o.P = P;
            o.D = reflect64(I, N, c);
            return;
        }
        R = snell64(I, N, mu, c, D);
        n_last = n_in;
        Delta = t.dL0 / n_in;
        decide = false;
    }
    for (;;) {
        if (decide) {
            double ni;
            d3 g;
            med64<MK>(m, P, ni, g);
            double gl = sqrt(dot(g, g));
            if (!isfinite(gl) || gl == 0.0) {  // cases (ii)/(iii)
                R = I;
                Delta = t.dL0 / ni;
                o.flags |= VRT_FLAG_STRAIGHT;
            } else {
                d3 N = mk(g.x / gl, g.y / gl, g.z / gl);  // Eq. (5)
                double c = dot(N, I);
                if (fabs(c) <= t.eps_tan) {  // case (iv), Eqs. (16)-(18)
                    Delta = t.dL0 / ni;
                    double dn = index64<MK>(m, P + Delta * N) - ni;
                    double a = dn / (2.0 * ni);
                    double w = 1.0 - a * a;
                    d3 v = sqrt(w > 0.0 ? w : 0.0) * I + a * N;
                    double lv = sqrt(dot(v, v));
                    R = mk(v.x / lv, v.y / lv, v.z / lv);
                    o.flags |= VRT_FLAG_TANGENT;
                } else {
                    double mu = n_last / ni;
                    double D = 1.0 - mu * mu * (1.0 - c * c);
                    if (near_critical(mu, c, D, t.crit_rad)) o.flags |= VRT_FLAG_NEAR_CRITICAL;
                    if (mu < 1.0 && fabs(c) < t.crit_rad) o.flags |= VRT_FLAG_NEAR_GRAZING;
                    if (D <= 0.0) {  // case (v), Eqs. (19)-(20)
                        R = reflect64(I, N, c);
                        Delta = t.dL0 / n_last;
                        o.ntir++;
                    } else {
                        R = snell64(I, N, mu, c, D);
                        Delta = t.dL0 / ni;
                    }
                }
            }
            n_last = ni;
        }
        decide = true;
        for (;;) {  // move along R, possibly meeting the surface
            int face;
            double tx = surf_exit(b, P, R, face);
            o.steps++;
            if (tx < 3.0 * Delta) {  // distance of the step end from the surface
                const d3 Ne = surf_normal(b, P + tx * R, face);
                if (fabs(tx - Delta) * fabs(dot(R, Ne)) < t.tie_eps) o.flags |= VRT_FLAG_NEAR_TIE;
            }
            if (tx > Delta) {
                P = P + Delta * R;
                I = R;
                path.add(P);
                if ((int64_t)o.steps >= t.max_steps) {
                    o.status = VRT_RAY_TRUNCATED;
                    o.P = P;
                    o.D = I;
                    return;
                }
                break;
            }
            P = P + tx * R;
            surf_snap(b, P, face);
            path.add(P);
            d3 N = surf_normal(b, P, face);
            double mu = n_last / m.n_amb, c = dot(N, R);
            double D = 1.0 - mu * mu * (1.0 - c * c);
            if (near_critical(mu, c, D, t.crit_rad)) o.flags |= VRT_FLAG_NEAR_CRITICAL;
            if (D <= 0.0) {  // reflected back inside at the surface
                R = reflect64(R, N, c);
                Delta = t.dL0 / n_last;
                n_last = index64<MK>(m, P);
                o.nbtir++;
                o.flags |= VRT_FLAG_BOUNDARY_TIR;
                if ((int64_t)o.steps >= t.max_steps) {
                    o.status = VRT_RAY_TRUNCATED;
                    o.P = P;
                    o.D = R;
                    return;
                }
                continue;
            }
            d3 Ro = snell64(R, N, mu, c, D);
            o.P = P;
            o.D = Ro;
            o.status = VRT_RAY_EXITED;
            if (t.has_plane) {
                if (!(Ro.z > 0.0) || (t.plane_z - P.z) / Ro.z < 0.0) {
                    o.status = VRT_RAY_NO_PLANE;
                } else {
                    double s = (t.plane_z - P.z) / Ro.z;
                    o.P = mk(P.x + s * Ro.x, P.y + s * Ro.y, t.plane_z);
                }
            }
            return;
        }
    }
}

template <int MK>
__device__ __forceinline__ void trace_ray64(const MediumDev &m, const BoundaryDev &b,
                                            const TraceDev &t, d3 P0, d3 d0, Out64 &o) {
    NoPath none;
    trace_ray64<MK>(m, b, t, P0, d0, o, none);
}

}  // namespace vrt
