// vrt_common.h -- internal definitions shared by the HIP sources of libvrt.
//
// Device-side descriptions of a medium, its enclosing surface and a trace
// request, small vector helpers, and the geometry of the enclosing surface
// (inside test, entry / exit distances, outward normals).  All surface
// geometry is double precision: it runs once per surface event, not per step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vrt.h"

namespace vrt {

// ---------------------------------------------------------------------------
// descriptors passed by value to kernels
// ---------------------------------------------------------------------------
struct BoundaryDev {
    int kind;  // vrt_boundary_kind
    double p[6];
    float pf[6];  // the same parameters rounded to float (per-step inside test)
};

// Per-bump single-precision record of the Gaussian-sum medium (10 floats):
// A, -log2(e)/(2 sigma^2), cx, cy, cz, then the Taylor coefficients of
// A expm1(y / sigma^2) in y:  A/sigma^2, A/(2 sigma^4), A/(6 sigma^6),
// A/(24 sigma^8), A/(120 sigma^10).  The double record is the raw
// (A, sigma, cx, cy, cz).
constexpr int kBumpF = 10;
constexpr int kBumpD = 5;

// Fill one single-precision bump record from (A, sigma, cx, cy, cz).
__host__ __device__ inline void fill_bump_f(const double *q, float *o) {
    const double is2 = 1.0 / (q[1] * q[1]);
    o[0] = (float)q[0];
    o[1] = (float)(-0.5 * is2 / 0.69314718055994530942);  // -log2(e) / (2 sigma^2)
    o[2] = (float)q[2];
    o[3] = (float)q[3];
    o[4] = (float)q[4];
    double c = q[0];
    const double fact[5] = {1.0, 2.0, 6.0, 24.0, 120.0};
    for (int j = 0; j < 5; ++j) {
        c *= is2;
        o[5 + j] = (float)(c / fact[j]);
    }
}

struct MediumDev {
    int kind;        // vrt_medium_kind
    int K;           // bumps (GAUSSIAN); mask of the Fringe terms present (ZERNIKE)
    double n_amb;    // surroundings
    double q[8];     // analytic parameters as given (layout in media.h)
    const double *bumps_d;  // K * kBumpD (GAUSSIAN); 16 x 4 coefficient table (ZERNIKE)
    const float *bumps_f;   // K * kBumpF (GAUSSIAN)
    // discretized medium
    const float *grid;      // nz*ny*nx node values, x fastest
    const float4 *rec;      // nz*ny*nx node records (n, h_x, h_y, h_z), see media.h
    int rec_exact;          // every h_a is the exact node difference over its spacings
    int nx, ny, nz;
    double lo[3], hi[3], h[3], inv_h[3];
    float flo[3], fhi[3], finv_h[3];
};

struct TraceDev {
    double dL0;
    int64_t max_steps;
    double eps_tan;
    double crit_rad;
    double tie_eps;
    double plane_z;
    int has_plane;
};

template <typename T>
struct RaysDev {
    const T *px, *py, *pz, *dx, *dy, *dz;
    T *ox, *oy, *oz, *odx, *ody, *odz;
    uint32_t *status, *steps, *n_tir, *n_btir, *flags;
};

// face ids: box 0..5 = (x lo, y lo, z lo, x hi, y hi, z hi); sphere 7;
// cylinder: 6 side, 2 bottom (z0), 5 top (z1)
constexpr int kFaceSphere = 7;
constexpr int kFaceSide = 6;

// ---------------------------------------------------------------------------
// vector helpers
// ---------------------------------------------------------------------------
struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 mk(double x, double y, double z) { return d3{x, y, z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double get(d3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
__device__ __forceinline__ void set(d3 &a, int i, double v) {
    if (i == 0) a.x = v;
    else if (i == 1) a.y = v;
    else a.z = v;
}

struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mkf(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ float dotf(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// ---------------------------------------------------------------------------
// enclosing surface (Sec. II case (i)); convex: box, sphere, z-cylinder
// ---------------------------------------------------------------------------
__device__ inline bool surf_inside_strict(const BoundaryDev &b, d3 P) {
    if (b.kind == VRT_BOUNDARY_BOX)
        return P.x > b.p[0] && P.x < b.p[3] && P.y > b.p[1] && P.y < b.p[4] && P.z > b.p[2] &&
               P.z < b.p[5];
    if (b.kind == VRT_BOUNDARY_SPHERE) {
        d3 o = P - mk(b.p[0], b.p[1], b.p[2]);
        return dot(o, o) < b.p[3] * b.p[3];
    }
    double x = P.x - b.p[0], y = P.y - b.p[1];
    return x * x + y * y < b.p[2] * b.p[2] && P.z > b.p[3] && P.z < b.p[4];
}

// Where a ray from outside (or on) the surface first enters the interior.
// Returns false when the line misses it; a line that only touches misses.
__device__ inline bool surf_entry(const BoundaryDev &b, d3 P, d3 d, double &t, int &face) {
    if (b.kind == VRT_BOUNDARY_BOX) {
        double tn = -INFINITY, tf = INFINITY;
        int fn = -1;
        for (int a = 0; a < 3; ++a) {
            double pa = get(P, a), da = get(d, a), lo = b.p[a], hi = b.p[a + 3];
            if (da == 0.0) {
                if (pa < lo || pa > hi) return false;
                continue;
            }
            double tl = (lo - pa) / da, th = (hi - pa) / da;
            int fl = a, fh = a + 3;
            double t0 = tl < th ? tl : th, t1 = tl < th ? th : tl;
            int f0 = tl < th ? fl : fh;
            if (t0 > tn) {
                tn = t0;
                fn = f0;
            }
            if (t1 < tf) tf = t1;
        }
        if (fn < 0 || !(tn < tf) || tn < 0.0) return false;
        t = tn;
        face = fn;
        return true;
    }
    if (b.kind == VRT_BOUNDARY_SPHERE) {
        d3 o = P - mk(b.p[0], b.p[1], b.p[2]);
        double bb = dot(o, d), cc = dot(o, o) - b.p[3] * b.p[3];
        double disc = bb * bb - cc;
        if (!(disc > 0.0)) return false;
        double t1 = -bb - sqrt(disc);
        if (t1 < 0.0) return false;
        t = t1;
        face = kFaceSphere;
        return true;
    }
    // z-cylinder: side interval intersected with the z slab
    double x = P.x - b.p[0], y = P.y - b.p[1], r = b.p[2];
    double a2 = d.x * d.x + d.y * d.y, bb = x * d.x + y * d.y, cc = x * x + y * y - r * r;
    double s0, s1;
    if (a2 == 0.0) {
        if (!(cc < 0.0)) return false;
        s0 = -INFINITY;
        s1 = INFINITY;
    } else {
        double disc = bb * bb - a2 * cc;
        if (!(disc > 0.0)) return false;
        double sq = sqrt(disc);
        s0 = (-bb - sq) / a2;
        s1 = (-bb + sq) / a2;
    }
    double z0, z1;
    int fz0;
    if (d.z == 0.0) {
        if (P.z < b.p[3] || P.z > b.p[4]) return false;
        z0 = -INFINITY;
        z1 = INFINITY;
        fz0 = -1;
    } else {
        double ta = (b.p[3] - P.z) / d.z, tb = (b.p[4] - P.z) / d.z;
        z0 = ta < tb ? ta : tb;
        z1 = ta < tb ? tb : ta;
        fz0 = ta < tb ? 2 : 5;
    }
    double tn, tf = s1 < z1 ? s1 : z1;
    int fn;
    if (s0 >= z0) {
        tn = s0;
        fn = kFaceSide;
    } else {
        tn = z0;
        fn = fz0;
    }
    if (!(tn < tf) || tn < 0.0 || fn < 0) return false;
    t = tn;
    face = fn;
    return true;
}

// Distance from a point inside (or on) the surface along unit R to the
// surface, and the face reached (planar ties -> lower axis index).
__device__ inline double surf_exit(const BoundaryDev &b, d3 P, d3 R, int &face) {
    if (b.kind == VRT_BOUNDARY_BOX) {
        double best = INFINITY;
        int bf = 0;
        for (int a = 0; a < 3; ++a) {
            double ra = get(R, a);
            if (ra == 0.0) continue;
            double t = ra > 0.0 ? (b.p[a + 3] - get(P, a)) / ra : (b.p[a] - get(P, a)) / ra;
            if (t < best) {
                best = t;
                bf = ra > 0.0 ? a + 3 : a;
            }
        }
        face = bf;
        return best > 0.0 ? best : 0.0;
    }
    if (b.kind == VRT_BOUNDARY_SPHERE) {
        d3 o = P - mk(b.p[0], b.p[1], b.p[2]);
        double bb = dot(o, R), cc = dot(o, o) - b.p[3] * b.p[3];
        double disc = bb * bb - cc;
        double t = -bb + sqrt(disc > 0.0 ? disc : 0.0);
        face = kFaceSphere;
        return t > 0.0 ? t : 0.0;
    }
    double x = P.x - b.p[0], y = P.y - b.p[1], r = b.p[2];
    double a2 = R.x * R.x + R.y * R.y;
    double best = INFINITY;
    int bf = kFaceSide;
    if (a2 > 0.0) {
        double bb = x * R.x + y * R.y, cc = x * x + y * y - r * r;
        double disc = bb * bb - a2 * cc;
        best = (-bb + sqrt(disc > 0.0 ? disc : 0.0)) / a2;
    }
    if (R.z != 0.0) {
        double t = R.z > 0.0 ? (b.p[4] - P.z) / R.z : (b.p[3] - P.z) / R.z;
        if (t < best) {
            best = t;
            bf = R.z > 0.0 ? 5 : 2;
        }
    }
    face = bf;
    return best > 0.0 ? best : 0.0;
}

// Put a point reached on a planar face exactly on that face.
__device__ inline void surf_snap(const BoundaryDev &b, d3 &P, int face) {
    if (b.kind == VRT_BOUNDARY_BOX) {
        set(P, face % 3, b.p[face]);
    } else if (b.kind == VRT_BOUNDARY_CYLINDER) {
        if (face == 2) P.z = b.p[3];
        if (face == 5) P.z = b.p[4];
    }
}

__device__ inline d3 surf_normal(const BoundaryDev &b, d3 P, int face) {
    if (b.kind == VRT_BOUNDARY_BOX) {
        d3 N = mk(0, 0, 0);
        set(N, face % 3, face < 3 ? -1.0 : 1.0);
        return N;
    }
    if (b.kind == VRT_BOUNDARY_SPHERE) {
        const d3 o = P - mk(b.p[0], b.p[1], b.p[2]);
        const double r = sqrt(dot(o, o));
        return mk(o.x / r, o.y / r, o.z / r);
    }
    if (face == 2) return mk(0, 0, -1.0);
    if (face == 5) return mk(0, 0, 1.0);
    double x = P.x - b.p[0], y = P.y - b.p[1];
    double rr = sqrt(x * x + y * y);
    return mk(x / rr, y / rr, 0.0);
}

// Strictly inside with a margin (single precision fast test of a step end).
__device__ __forceinline__ bool surf_inside_margin(const BoundaryDev &b, float x, float y, float z,
                                                   float mrg) {
    const float *q = b.pf;
    if (b.kind == VRT_BOUNDARY_BOX)
        return x > q[0] + mrg && x < q[3] - mrg && y > q[1] + mrg && y < q[4] - mrg &&
               z > q[2] + mrg && z < q[5] - mrg;
    if (b.kind == VRT_BOUNDARY_SPHERE) {
        float ox = x - q[0], oy = y - q[1], oz = z - q[2];
        float r = q[3] - mrg;
        return ox * ox + oy * oy + oz * oz < r * r;
    }
    float ox = x - q[0], oy = y - q[1];
    float r = q[2] - mrg;
    return ox * ox + oy * oy < r * r && z > q[3] + mrg && z < q[4] - mrg;
}

// ---------------------------------------------------------------------------
// local vectorial rules in double precision
// ---------------------------------------------------------------------------
// Near-critical test: mu > 1 and |acos|c| - asin(1/mu)| < eps.  |D| >=
// 2 mu^2 eps excludes it without trigonometry (D = mu^2 (cos a - cos b)
// (cos a + cos b) and |cos a - cos b| <= |a - b|).
__device__ inline bool near_critical(double mu, double c, double D, double eps) {
    if (!(mu > 1.0) || !(eps > 0.0)) return false;
    if (fabs(D) >= 2.0 * mu * mu * eps) return false;
    double ac = fabs(c);
    ac = ac > 1.0 ? 1.0 : ac;
    return fabs(acos(ac) - asin(1.0 / mu)) < eps;
}

// Eq. (20) direction: I - 2 (I.N) N, normalised.
__device__ inline d3 reflect64(d3 I, d3 N, double c) {
    const d3 v = I - (2.0 * c) * N;
    const double l = sqrt(dot(v, v));
    return mk(v.x / l, v.y / l, v.z / l);
}

// Eqs. (9)-(10), "+" root.
__device__ inline d3 snell64(d3 I, d3 N, double mu, double c, double D) {
    double g = -mu * c + (c > 0.0 ? 1.0 : -1.0) * sqrt(D);
    return mu * I + g * N;
}

}  // namespace vrt
