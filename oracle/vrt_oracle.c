/*
 * vrt_oracle.c -- plain FP64 CPU oracle of the vectorial ray tracing (VRT)
 * march of "Generalized vectorial ray tracing for optical analysis and design
 * in freeform gradient-index media".
 *
 * TEST INFRASTRUCTURE ONLY.  It exists to check the GPU library; nothing in
 * the product path may call it.  It is deliberately slow and literal: one ray
 * at a time, IEEE double, no fast-math, no FMA contraction
 * (-ffp-contract=off), each step written in the order the paper gives it.
 * Parallelism is only across independent rays (OpenMP).
 *
 * What it computes (per ray), with the readings taken where the paper is
 * silent:
 *   - launch direction I_0 = d0/|d0| (Sec. II, flowchart caption gives I_0 as a
 *     unit vector built from (theta0, phi0));
 *   - a ray that starts outside the medium travels straight in the homogeneous
 *     surroundings (case (iii), Eq. (12)) to its exact intersection with the
 *     enclosing surface and is refracted there with the surface normal
 *     (case (i)) using Eqs. (9)-(10) with mu = n_amb / n(P_B);
 *   - inside, every step evaluates n and grad n at P_i (Eq. (5)) and applies,
 *     in this order: undefined / zero gradient -> straight step (cases (ii),
 *     (iii), Eqs. (11)-(12)); tangential incidence N.I = 0 -> circular-arc rule
 *     (case (iv), Eqs. (16)-(18)); TIR when mu^2 (1 - (N.I)^2) >= 1 (case (v),
 *     Eqs. (19)-(20)); otherwise vectorial Snell (Eqs. (9)-(10), "+" root);
 *   - the position advances by Delta_i = dL0 / n_i (Eqs. (3)-(4)), or by
 *     Delta_{i-1} = dL0 / n_{i-1} after a TIR (Eq. (20)); as Sec. II states,
 *     n_{i-1} = n(P_{i-1}) is the index at the previous point of the polyline
 *     and n_i = n(P_i) the index at the point where the ray is refracted;
 *   - a step that would cross the enclosing surface is cut at the exact
 *     intersection P_B, which becomes a point of the polyline; there Snell with
 *     the surface normal (case (i)) and mu = n(P_{i-1}) / n_amb either
 *     transmits the ray (EXITED) or reflects it (boundary TIR: the ray stays
 *     inside and moves on from P_B with dL0 / n(P_{i-1}));
 *   - every decision with mu > 1 is checked against the critical angle and
 *     flagged when |acos|N.I| - asin(1/mu)| < crit_rad; a refraction with
 *     mu < 1 at |N.I| < crit_rad is flagged as near grazing (the sgn(N.I) of
 *     Eq. (10) puts the refracted ray on one side of the isoindicial surface
 *     or the other); a move whose end lies within tie_eps of the enclosing
 *     surface, measured perpendicular to it, is flagged as a near tie (the
 *     choice "full step or cut at the surface" is then decided by rounding).
 *     Each of the three windows is also checked ten times wider (flag bits
 *     64, 128, 256): a decision that close may still go either way once the
 *     state carries the rounding of a single-precision march.
 * The incident direction I_i is carried as the previous R (Eq. (6) gives the
 * same vector in exact arithmetic).
 */
#include "vrt_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------ */
/* medium: n(P) and grad n(P)                                           */
/* ------------------------------------------------------------------ */
static double grid_node(const orc_medium *m, int i, int j, int k) {
    return (double)m->grid[((size_t)k * m->ny + j) * m->nx + i];
}

/* Central difference of the node values along one axis, one-sided at the
 * first and last node (trilinear-grid reading of a discretized medium). */
static double grid_node_diff(const orc_medium *m, int i, int j, int k, int axis, double h) {
    int idx[3] = {i, j, k};
    int nn[3] = {m->nx, m->ny, m->nz};
    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
    double span;
    if (idx[axis] == 0) {
        hi[axis] = 1;
        span = h;
    } else if (idx[axis] == nn[axis] - 1) {
        lo[axis] = nn[axis] - 2;
        span = h;
    } else {
        lo[axis] = idx[axis] - 1;
        hi[axis] = idx[axis] + 1;
        span = 2.0 * h;
    }
    return (grid_node(m, hi[0], hi[1], hi[2]) - grid_node(m, lo[0], lo[1], lo[2])) / span;
}

static void grid_eval(const orc_medium *m, const double P[3], double *n, double g[3]) {
    int nn[3] = {m->nx, m->ny, m->nz};
    int cell[3];
    double f[3], h[3];
    for (int a = 0; a < 3; ++a) {
        h[a] = (m->ghi[a] - m->glo[a]) / (double)(nn[a] - 1);
        double x = P[a];
        if (x < m->glo[a]) x = m->glo[a];
        if (x > m->ghi[a]) x = m->ghi[a];
        double u = (x - m->glo[a]) / h[a];
        int c = (int)floor(u);
        if (c < 0) c = 0;
        if (c > nn[a] - 2) c = nn[a] - 2;
        cell[a] = c;
        f[a] = u - (double)c;
    }
    *n = 0.0;
    g[0] = g[1] = g[2] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                           (dz ? f[2] : 1.0 - f[2]);
                int i = cell[0] + dx, j = cell[1] + dy, k = cell[2] + dz;
                *n += w * grid_node(m, i, j, k);
                for (int a = 0; a < 3; ++a) g[a] += w * grid_node_diff(m, i, j, k, a, h[a]);
            }
}

/* Fringe Zernike polynomial j (1-based Fringe ordering; j <= 16) as
 * (radial order n, azimuthal order m, cosine or sine). */
static const int fringe_nm[17][3] = {
    {0, 0, 0}, {0, 0, 0}, {1, 1, 0}, {1, 1, 1}, {2, 0, 0}, {2, 2, 0}, {2, 2, 1},
    {3, 1, 0}, {3, 1, 1}, {4, 0, 0}, {3, 3, 0}, {3, 3, 1}, {4, 2, 0}, {4, 2, 1},
    {5, 1, 0}, {5, 1, 1}, {6, 0, 0}};

static double fact(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* Radial polynomial R_n^m(rho) = sum_k (-1)^k (n-k)! / (k! ((n+m)/2-k)! ((n-m)/2-k)!)
 * rho^(n-2k), its derivative, and R / rho (m >= 1, a polynomial). */
static void zernike_radial(int n, int m, double rho, double *R, double *dR, double *Rr) {
    *R = *dR = *Rr = 0.0;
    for (int k = 0; k <= (n - m) / 2; ++k) {
        double c = ((k % 2) ? -1.0 : 1.0) * fact(n - k) /
                   (fact(k) * fact((n + m) / 2 - k) * fact((n - m) / 2 - k));
        int e = n - 2 * k;
        *R += c * pow(rho, e);
        if (e >= 1) *dR += c * e * pow(rho, e - 1);
        if (e >= 1) *Rr += c * pow(rho, e - 1);
    }
}

/* Legendre P_l(w) and P_l'(w) by the three-term recursion. */
static void legendre(int l, double w, double *P, double *dP) {
    double p0 = 1.0, p1 = w, d0 = 0.0, d1 = 1.0;
    if (l == 0) {
        *P = 1.0;
        *dP = 0.0;
        return;
    }
    for (int k = 1; k < l; ++k) {
        double p2 = ((2 * k + 1) * w * p1 - k * p0) / (k + 1);
        double d2 = d0 + (2 * k + 1) * p1;
        p0 = p1;
        p1 = p2;
        d0 = d1;
        d1 = d2;
    }
    *P = p1;
    *dP = d1;
}

static void medium_eval(const orc_medium *m, const double P[3], double *n, double g[3]) {
    const double *p = m->params;
    switch (m->kind) {
    case ORC_HOMOGENEOUS:
        *n = p[0];
        g[0] = g[1] = g[2] = 0.0;
        return;
    case ORC_LINEAR:
        *n = p[0] + p[1] * P[0] + p[2] * P[1] + p[3] * P[2];
        g[0] = p[1];
        g[1] = p[2];
        g[2] = p[3];
        return;
    case ORC_LUNEBURG: {
        /* n = sqrt(2 - r^2/R^2); grad n = -(P - C) / (R^2 n) */
        double R = p[0];
        double d[3] = {P[0] - p[1], P[1] - p[2], P[2] - p[3]};
        double nv = sqrt(2.0 - dot3(d, d) / (R * R));
        *n = nv;
        for (int a = 0; a < 3; ++a) g[a] = -d[a] / (R * R * nv);
        return;
    }
    case ORC_FIBER: {
        /* Eq. (21): n^2 = n_c^2 (1 - 2 Delta rho^2 / R^2) in the core,
         * n_c^2 (1 - 2 Delta) in the cladding rho > R */
        double nc = p[0], Dl = p[1], R = p[2];
        double x = P[0] - p[3], y = P[1] - p[4];
        double rho2 = x * x + y * y;
        if (rho2 <= R * R) {
            double nv = nc * sqrt(1.0 - 2.0 * Dl * rho2 / (R * R));
            *n = nv;
            double k = -2.0 * Dl * nc * nc / (R * R * nv);
            g[0] = k * x;
            g[1] = k * y;
            g[2] = 0.0;
        } else {
            *n = nc * sqrt(1.0 - 2.0 * Dl);
            g[0] = g[1] = g[2] = 0.0;
        }
        return;
    }
    case ORC_GAUSSIAN: {
        /* n = n0 + sum_k A_k exp(-|P - c_k|^2 / (2 sigma_k^2)) */
        int K = (int)p[1];
        double nv = p[0];
        g[0] = g[1] = g[2] = 0.0;
        for (int k = 0; k < K; ++k) {
            const double *b = p + 2 + 5 * k;
            double A = b[0], s = b[1];
            double d[3] = {P[0] - b[2], P[1] - b[3], P[2] - b[4]};
            double e = A * exp(-dot3(d, d) / (2.0 * s * s));
            nv += e;
            for (int a = 0; a < 3; ++a) g[a] += -e * d[a] / (s * s);
        }
        *n = nv;
        return;
    }
    case ORC_GRID:
        grid_eval(m, P, n, g);
        return;
    case ORC_SPHERICAL: {
        /* Sec. V, Eq. (26): n = a0 + a1 G1 + a2 G2 + a3 G3 in spherical
         * coordinates (r, theta, phi) about the centre c, theta measured from
         * the z axis:  G1 = 0.3 (r^2 - 1),  G2 = r cos(5 theta),
         * G3 = r^2 sin^2(theta) cos(2 phi).  The gradient is
         * dn/dr r^ + (1/r) dn/dtheta theta^ + 1/(r sin theta) dn/dphi phi^.
         * At r = 0 the direction of G2's gradient is undefined (a cusp): the
         * gradient is returned as NaN there, which the march takes as case (ii). */
        double a0 = p[0], a1 = p[1], a2 = p[2], a3 = p[3];
        double x = P[0] - p[4], y = P[1] - p[5], z = P[2] - p[6];
        double r = sqrt(x * x + y * y + z * z);
        if (r == 0.0) {
            *n = a0 - 0.3 * a1;
            g[0] = g[1] = g[2] = NAN;
            return;
        }
        double th = acos(fmax(-1.0, fmin(1.0, z / r)));
        double ph = atan2(y, x);
        double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
        double G1 = 0.3 * (r * r - 1.0);
        double G2 = r * cos(5.0 * th);
        double G3 = r * r * st * st * cos(2.0 * ph);
        *n = a0 + a1 * G1 + a2 * G2 + a3 * G3;
        /* components along r^, theta^, phi^ */
        double dr = a1 * 0.6 * r + a2 * cos(5.0 * th) + a3 * 2.0 * r * st * st * cos(2.0 * ph);
        double dt = a2 * (-5.0 * sin(5.0 * th)) + a3 * 2.0 * r * st * ct * cos(2.0 * ph);
        double dp = a3 * (-2.0 * r * st * sin(2.0 * ph));
        double er[3] = {st * cp, st * sp, ct};
        double et[3] = {ct * cp, ct * sp, -st};
        double ep[3] = {-sp, cp, 0.0};
        for (int a = 0; a < 3; ++a) g[a] = dr * er[a] + dt * et[a] + dp * ep[a];
        return;
    }
    case ORC_ZERNIKE: {
        /* Sec. V: n = n0 + dn sum c_{j,l} Z_j(x', y') V_l(z'), x' = x / rho_max,
         * y' = y / rho_max, z' = 2 z / z_max - 1, n0 = (n_hi + n_lo) / 2,
         * dn = (n_hi - n_lo) / 2; Z_j Fringe Zernike polynomials in polar form
         * R(rho) cos/sin(m theta), V_l Legendre polynomials. */
        double nlo = p[0], nhi = p[1], rm = p[2], zm = p[3];
        int K = (int)p[4];
        double n0 = 0.5 * (nhi + nlo), dn = 0.5 * (nhi - nlo);
        double u = P[0] / rm, v = P[1] / rm, w = 2.0 * P[2] / zm - 1.0;
        double rho = sqrt(u * u + v * v), th = atan2(v, u);
        double ct = cos(th), st = sin(th);
        double nv = n0;
        g[0] = g[1] = g[2] = 0.0;
        for (int k = 0; k < K; ++k) {
            int j = (int)p[5 + 3 * k], l = (int)p[6 + 3 * k];
            double c = p[7 + 3 * k];
            int rn = fringe_nm[j][0], am = fringe_nm[j][1], sn = fringe_nm[j][2];
            double R, dR, Rr;
            zernike_radial(rn, am, rho, &R, &dR, &Rr);
            double T = am == 0 ? 1.0 : (sn ? sin(am * th) : cos(am * th));
            double dT = am == 0 ? 0.0 : (sn ? am * cos(am * th) : -am * sin(am * th));
            double Z = R * T;
            double Zu = dR * ct * T - Rr * dT * st; /* d/du = cos d/drho - sin/rho d/dtheta */
            double Zv = dR * st * T + Rr * dT * ct;
            double V, dV;
            legendre(l, w, &V, &dV);
            nv += dn * c * Z * V;
            g[0] += dn * c * Zu * V / rm;
            g[1] += dn * c * Zv * V / rm;
            g[2] += dn * c * Z * dV * 2.0 / zm;
        }
        *n = nv;
        return;
    }
    case ORC_N2P: {
        /* Sec. VI, Eq. (27): n = [1 + ((R^2 - (rho/2)^2) / F^2)^beta]^gamma inside
         * the lens (rho = distance from the z axis); the lens volume
         * (0 <= rho <= R, -L <= z <= 0) is the enclosing cylinder and n = 1 the
         * surroundings.  dn/drho = gamma [1 + w^beta]^(gamma - 1) beta w^(beta - 1)
         * dw/drho with w = (R^2 - rho^2/4) / F^2, dw/drho = -rho / (2 F^2). */
        double R = p[0], F = p[1], be = p[2], ga = p[3];
        double x = P[0], y = P[1];
        double rho = sqrt(x * x + y * y);
        double w = (R * R - (rho / 2.0) * (rho / 2.0)) / (F * F);
        double u = 1.0 + pow(w, be);
        *n = pow(u, ga);
        double dndrho = ga * pow(u, ga - 1.0) * be * pow(w, be - 1.0) * (-rho / (2.0 * F * F));
        if (rho == 0.0) {
            g[0] = g[1] = g[2] = 0.0;
        } else {
            g[0] = dndrho * x / rho;
            g[1] = dndrho * y / rho;
            g[2] = 0.0;
        }
        return;
    }
    default:
        *n = NAN;
        g[0] = g[1] = g[2] = NAN;
    }
}

static double medium_index(const orc_medium *m, const double P[3]) {
    double n, g[3];
    medium_eval(m, P, &n, g);
    return n;
}

/* ------------------------------------------------------------------ */
/* enclosing surface                                                    */
/* ------------------------------------------------------------------ */
static int inside_strict(const orc_medium *m, const double P[3]) {
    const double *b = m->bparams;
    switch (m->bkind) {
    case ORC_BOX:
        return P[0] > b[0] && P[0] < b[3] && P[1] > b[1] && P[1] < b[4] && P[2] > b[2] &&
               P[2] < b[5];
    case ORC_SPHERE: {
        double d[3] = {P[0] - b[0], P[1] - b[1], P[2] - b[2]};
        return dot3(d, d) < b[3] * b[3];
    }
    case ORC_CYLINDER: {
        double x = P[0] - b[0], y = P[1] - b[1];
        return x * x + y * y < b[2] * b[2] && P[2] > b[3] && P[2] < b[4];
    }
    }
    return 0;
}

/* Face ids used to put a boundary point exactly on a planar face:
 * box: 0..5 = (x lo, y lo, z lo, x hi, y hi, z hi); cylinder: 6 = side,
 * 2 = z0 plane, 5 = z1 plane; sphere: 7. */
static void snap_to_face(const orc_medium *m, double P[3], int face) {
    const double *b = m->bparams;
    if (m->bkind == ORC_BOX) {
        P[face % 3] = b[face];
    } else if (m->bkind == ORC_CYLINDER) {
        if (face == 2) P[2] = b[3];
        if (face == 5) P[2] = b[4];
    }
}

static void outward_normal(const orc_medium *m, const double P[3], int face, double N[3]) {
    const double *b = m->bparams;
    N[0] = N[1] = N[2] = 0.0;
    if (m->bkind == ORC_BOX) {
        N[face % 3] = face < 3 ? -1.0 : 1.0;
    } else if (m->bkind == ORC_SPHERE) {
        double d[3] = {P[0] - b[0], P[1] - b[1], P[2] - b[2]};
        double r = norm3(d);
        for (int a = 0; a < 3; ++a) N[a] = d[a] / r;
    } else {
        if (face == 2) {
            N[2] = -1.0;
        } else if (face == 5) {
            N[2] = 1.0;
        } else {
            double x = P[0] - b[0], y = P[1] - b[1];
            double r = sqrt(x * x + y * y);
            N[0] = x / r;
            N[1] = y / r;
        }
    }
}

/* Entry of a ray that starts outside (or on) the surface.  Returns 1 and the
 * parameter t >= 0 and the face of the first crossing into the interior, or 0
 * when the line misses the interior (touching counts as a miss). */
static int entry_hit(const orc_medium *m, const double P[3], const double d[3], double *t,
                     int *face) {
    const double *b = m->bparams;
    if (m->bkind == ORC_BOX) {
        double tn = -INFINITY, tf = INFINITY;
        int fn = -1;
        for (int a = 0; a < 3; ++a) {
            if (d[a] == 0.0) {
                if (P[a] < b[a] || P[a] > b[a + 3]) return 0;
                continue;
            }
            double t0 = (b[a] - P[a]) / d[a], t1 = (b[a + 3] - P[a]) / d[a];
            int f0 = a, f1 = a + 3;
            if (t0 > t1) {
                double tt = t0;
                t0 = t1;
                t1 = tt;
                int ff = f0;
                f0 = f1;
                f1 = ff;
            }
            if (t0 > tn) {
                tn = t0;
                fn = f0;
            }
            if (t1 < tf) tf = t1;
        }
        if (fn < 0 || !(tn < tf) || tn < 0.0) return 0;
        *t = tn;
        *face = fn;
        return 1;
    }
    if (m->bkind == ORC_SPHERE) {
        double o[3] = {P[0] - b[0], P[1] - b[1], P[2] - b[2]};
        double bb = dot3(o, d), cc = dot3(o, o) - b[3] * b[3];
        double disc = bb * bb - cc;
        if (!(disc > 0.0)) return 0;
        double t1 = -bb - sqrt(disc);
        if (t1 < 0.0) return 0;
        *t = t1;
        *face = 7;
        return 1;
    }
    /* cylinder along z: intersect the side interval with the z slab */
    {
        double x = P[0] - b[0], y = P[1] - b[1];
        double a2 = d[0] * d[0] + d[1] * d[1];
        double bb = x * d[0] + y * d[1];
        double cc = x * x + y * y - b[2] * b[2];
        double ts0, ts1;
        if (a2 == 0.0) {
            if (!(cc < 0.0)) return 0;
            ts0 = -INFINITY;
            ts1 = INFINITY;
        } else {
            double disc = bb * bb - a2 * cc;
            if (!(disc > 0.0)) return 0;
            ts0 = (-bb - sqrt(disc)) / a2;
            ts1 = (-bb + sqrt(disc)) / a2;
        }
        double tz0, tz1;
        int fz0, fz1;
        if (d[2] == 0.0) {
            if (P[2] < b[3] || P[2] > b[4]) return 0;
            tz0 = -INFINITY;
            tz1 = INFINITY;
            fz0 = fz1 = -1;
        } else {
            double ta = (b[3] - P[2]) / d[2], tb = (b[4] - P[2]) / d[2];
            fz0 = 2;
            fz1 = 5;
            if (ta > tb) {
                double tt = ta;
                ta = tb;
                tb = tt;
                fz0 = 5;
                fz1 = 2;
            }
            tz0 = ta;
            tz1 = tb;
            (void)fz1;
        }
        double tn, tf = ts1 < tz1 ? ts1 : tz1;
        int fn;
        if (ts0 >= tz0) {
            tn = ts0;
            fn = 6;
        } else {
            tn = tz0;
            fn = fz0;
        }
        if (!(tn < tf) || tn < 0.0 || fn < 0) return 0;
        *t = tn;
        *face = fn;
        return 1;
    }
}

/* Distance from a point inside (or on) the surface along unit R to the
 * surface, and the face reached.  Ties between planar faces go to the lower
 * axis index. */
static double exit_dist(const orc_medium *m, const double P[3], const double R[3], int *face) {
    const double *b = m->bparams;
    if (m->bkind == ORC_BOX) {
        double best = INFINITY;
        int bf = 0;
        for (int a = 0; a < 3; ++a) {
            if (R[a] == 0.0) continue;
            double t = R[a] > 0.0 ? (b[a + 3] - P[a]) / R[a] : (b[a] - P[a]) / R[a];
            if (t < best) {
                best = t;
                bf = R[a] > 0.0 ? a + 3 : a;
            }
        }
        *face = bf;
        return best > 0.0 ? best : 0.0;
    }
    if (m->bkind == ORC_SPHERE) {
        double o[3] = {P[0] - b[0], P[1] - b[1], P[2] - b[2]};
        double bb = dot3(o, R), cc = dot3(o, o) - b[3] * b[3];
        double disc = bb * bb - cc;
        if (disc < 0.0) disc = 0.0;
        double t = -bb + sqrt(disc);
        *face = 7;
        return t > 0.0 ? t : 0.0;
    }
    {
        double x = P[0] - b[0], y = P[1] - b[1];
        double a2 = R[0] * R[0] + R[1] * R[1];
        double best = INFINITY;
        int bf = 6;
        if (a2 > 0.0) {
            double bb = x * R[0] + y * R[1];
            double cc = x * x + y * y - b[2] * b[2];
            double disc = bb * bb - a2 * cc;
            if (disc < 0.0) disc = 0.0;
            best = (-bb + sqrt(disc)) / a2;
        }
        if (R[2] != 0.0) {
            double t = R[2] > 0.0 ? (b[4] - P[2]) / R[2] : (b[3] - P[2]) / R[2];
            if (t < best) {
                best = t;
                bf = R[2] > 0.0 ? 5 : 2;
            }
        }
        *face = bf;
        return best > 0.0 ? best : 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* local vectorial rules                                                */
/* ------------------------------------------------------------------ */

/* Near-critical test: decisions with mu > 1 whose angle of incidence
 * acos|c| lies within eps of the critical angle asin(1/mu).  Since
 * D = mu^2 (cos(th_inc) - cos(th_c)) (cos(th_inc) + cos(th_c)) and cos is
 * 1-Lipschitz, |D| >= 2 mu^2 eps already rules the flag out, which spares the
 * trigonometry on almost every step without changing the answer. */
static int near_critical(double mu, double c, double D, double eps) {
    if (!(mu > 1.0) || !(eps > 0.0)) return 0;
    if (fabs(D) >= 2.0 * mu * mu * eps) return 0;
    double ac = fabs(c);
    if (ac > 1.0) ac = 1.0;
    double th_inc = acos(ac);
    double th_c = asin(1.0 / mu);
    return fabs(th_inc - th_c) < eps;
}

/* flag bits for a decision near the critical angle: the narrow window and the
 * ten times wider one */
static uint32_t critical_flags(double mu, double c, double D, double eps) {
    if (!near_critical(mu, c, D, 10.0 * eps)) return 0;
    return ORC_F_NEAR_CRITICAL_WIDE | (near_critical(mu, c, D, eps) ? ORC_F_NEAR_CRITICAL : 0);
}

/* Eq. (20): reflected unit direction I - 2 (I.N) N, normalised. */
static void reflect(const double I[3], const double N[3], double c, double R[3]) {
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = I[a] - 2.0 * c * N[a];
    double l = norm3(v);
    for (int a = 0; a < 3; ++a) R[a] = v[a] / l;
}

/* Eqs. (9)-(10), "+" root: R = mu I + gamma N,
 * gamma = -mu c + sgn(c) sqrt(1 - mu^2 (1 - c^2)), c = N.I != 0, D > 0. */
static void snell(const double I[3], const double N[3], double mu, double c, double D,
                  double R[3]) {
    double sg = c > 0.0 ? 1.0 : -1.0;
    double gamma = -mu * c + sg * sqrt(D);
    for (int a = 0; a < 3; ++a) R[a] = mu * I[a] + gamma * N[a];
}

/* ------------------------------------------------------------------ */
/* one ray                                                              */
/* ------------------------------------------------------------------ */
typedef struct {
    double *buf;
    int64_t cap, n;
} path_rec;

static void rec(path_rec *pr, const double P[3]) {
    if (!pr) return;
    if (pr->n < pr->cap) memcpy(pr->buf + 3 * pr->n, P, 3 * sizeof(double));
    pr->n++;
}

typedef struct {
    double P[3], D[3];
    uint32_t status, steps, ntir, nbtir, flags;
} ray_out;

static void finish_plane(const orc_params *q, ray_out *o) {
    if (!q->has_plane) return;
    /* straight continuation in the homogeneous surroundings to z = plane_z */
    double dz = o->D[2];
    if (!(dz > 0.0)) {
        o->status = ORC_NO_PLANE;
        return;
    }
    double t = (q->plane_z - o->P[2]) / dz;
    if (t < 0.0) {
        o->status = ORC_NO_PLANE;
        return;
    }
    o->P[0] += t * o->D[0];
    o->P[1] += t * o->D[1];
    o->P[2] = q->plane_z;
}

static void trace_one(const orc_medium *m, const orc_params *q, const double P0[3],
                      const double d0[3], ray_out *o, path_rec *pr) {
    double P[3], I[3], R[3], N[3];
    /* n_last = n at the most recent point of the polyline (n_{i-1} when the
     * ray is at P_i, Sec. II) */
    double n_last = 0.0, Delta = 0.0;
    int face;
    memset(o, 0, sizeof(*o));
    for (int a = 0; a < 3; ++a) {
        o->P[a] = P0[a];
        o->D[a] = d0[a];
    }
    {
        int ok = 1;
        for (int a = 0; a < 3; ++a) ok &= isfinite(P0[a]) && isfinite(d0[a]);
        double l = ok ? norm3(d0) : 0.0;
        if (!ok || !(l > 0.0)) {
            o->status = ORC_INVALID_INPUT;
            return;
        }
        for (int a = 0; a < 3; ++a) I[a] = d0[a] / l;
    }
    for (int a = 0; a < 3; ++a) P[a] = P0[a];
    rec(pr, P);

    if (inside_strict(m, P)) {
        /* a ray born inside: P0 is the previous point of the first step */
        n_last = medium_index(m, P);
        goto interior_step;
    } else {
        double t;
        if (!entry_hit(m, P, I, &t, &face)) {
            o->status = ORC_MISSED;
            for (int a = 0; a < 3; ++a) o->D[a] = I[a];
            return;
        }
        /* case (iii) in the surroundings: straight to the surface */
        for (int a = 0; a < 3; ++a) P[a] = P[a] + t * I[a];
        snap_to_face(m, P, face);
        rec(pr, P);
        outward_normal(m, P, face, N);
        double n_in = medium_index(m, P);
        double mu = m->n_amb / n_in;
        double c = dot3(N, I);
        double D = 1.0 - mu * mu * (1.0 - c * c);
        o->flags |= critical_flags(mu, c, D, q->crit_rad);
        if (D <= 0.0) {
            o->status = ORC_REFLECTED_AT_ENTRY;
            reflect(I, N, c, R);
            for (int a = 0; a < 3; ++a) {
                o->P[a] = P[a];
                o->D[a] = R[a];
            }
            return;
        }
        snell(I, N, mu, c, D, R);
        n_last = n_in;
        Delta = q->dL0 / n_in;
        goto move;
    }

interior_step:
    for (;;) {
        double ni, g[3];
        medium_eval(m, P, &ni, g);
        double gl = norm3(g);
        if (!isfinite(gl) || gl == 0.0) {
            /* cases (ii)/(iii): no defined normal -> straight, Eqs. (11)-(12) */
            for (int a = 0; a < 3; ++a) R[a] = I[a];
            Delta = q->dL0 / ni;
            o->flags |= ORC_F_STRAIGHT;
        } else {
            for (int a = 0; a < 3; ++a) N[a] = g[a] / gl; /* Eq. (5) */
            double c = dot3(N, I);
            if (fabs(c) <= q->eps_tan) {
                /* case (iv): arc of curvature grad n / n in the (I, N) plane,
                 * Eqs. (16)-(18), with Delta n from a probe at P + Delta N */
                Delta = q->dL0 / ni;
                double Pp[3];
                for (int a = 0; a < 3; ++a) Pp[a] = P[a] + Delta * N[a];
                double dn = medium_index(m, Pp) - ni;
                double h = dn / (2.0 * ni);
                double s = 1.0 - h * h;
                double w = sqrt(s > 0.0 ? s : 0.0);
                for (int a = 0; a < 3; ++a) R[a] = w * I[a] + h * N[a];
                double l = norm3(R);
                for (int a = 0; a < 3; ++a) R[a] /= l;
                o->flags |= ORC_F_TANGENT;
            } else {
                double mu = n_last / ni; /* mu_i = n_{i-1} / n_i */
                double D = 1.0 - mu * mu * (1.0 - c * c);
                o->flags |= critical_flags(mu, c, D, q->crit_rad);
                if (mu < 1.0 && fabs(c) < 10.0 * q->crit_rad) {
                    o->flags |= ORC_F_NEAR_GRAZING_WIDE;
                    if (fabs(c) < q->crit_rad) o->flags |= ORC_F_NEAR_GRAZING;
                }
                if (D <= 0.0) {
                    /* case (v): TIR, Eqs. (19)-(20) */
                    reflect(I, N, c, R);
                    Delta = q->dL0 / n_last;
                    o->ntir++;
                } else {
                    snell(I, N, mu, c, D, R);
                    Delta = q->dL0 / ni;
                }
            }
        }
        n_last = ni; /* P_i becomes the previous point of the next one */
    move:
        for (;;) {
            double tx = exit_dist(m, P, R, &face);
            o->steps++;
            if (tx < 3.0 * Delta) {
                /* distance of the step end from the surface, perpendicular to it */
                double Pe[3], Ne[3];
                for (int a = 0; a < 3; ++a) Pe[a] = P[a] + tx * R[a];
                outward_normal(m, Pe, face, Ne);
                double dist = fabs(tx - Delta) * fabs(dot3(R, Ne));
                if (dist < 10.0 * q->tie_eps) {
                    o->flags |= ORC_F_NEAR_TIE_WIDE;
                    if (dist < q->tie_eps) o->flags |= ORC_F_NEAR_TIE;
                }
            }
            if (tx > Delta) {
                /* Eq. (3) */
                for (int a = 0; a < 3; ++a) P[a] = P[a] + Delta * R[a];
                for (int a = 0; a < 3; ++a) I[a] = R[a];
                rec(pr, P);
                if ((int64_t)o->steps >= q->max_steps) {
                    o->status = ORC_TRUNCATED;
                    for (int a = 0; a < 3; ++a) {
                        o->P[a] = P[a];
                        o->D[a] = I[a];
                    }
                    return;
                }
                break; /* next interior step */
            }
            /* case (i): the step reaches the enclosing surface */
            for (int a = 0; a < 3; ++a) P[a] = P[a] + tx * R[a];
            snap_to_face(m, P, face);
            rec(pr, P);
            outward_normal(m, P, face, N);
            double mu = n_last / m->n_amb;
            double c = dot3(N, R);
            double D = 1.0 - mu * mu * (1.0 - c * c);
            o->flags |= critical_flags(mu, c, D, q->crit_rad);
            if (D <= 0.0) {
                double Rr[3];
                reflect(R, N, c, Rr);
                for (int a = 0; a < 3; ++a) R[a] = Rr[a];
                Delta = q->dL0 / n_last; /* Delta_{i-1}, Eq. (20) */
                n_last = medium_index(m, P); /* P_B is now the previous point */
                o->nbtir++;
                o->flags |= ORC_F_BOUNDARY_TIR;
                if ((int64_t)o->steps >= q->max_steps) {
                    o->status = ORC_TRUNCATED;
                    for (int a = 0; a < 3; ++a) {
                        o->P[a] = P[a];
                        o->D[a] = R[a];
                    }
                    return;
                }
                continue; /* move again from the boundary point */
            }
            {
                double Ro[3];
                snell(R, N, mu, c, D, Ro);
                o->status = ORC_EXITED;
                for (int a = 0; a < 3; ++a) {
                    o->P[a] = P[a];
                    o->D[a] = Ro[a];
                }
                finish_plane(q, o);
                return;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* exported                                                             */
/* ------------------------------------------------------------------ */
static int check_medium(const orc_medium *m, const orc_params *q) {
    if (!m || !q) return -1;
    if (!(q->dL0 > 0.0) || q->max_steps <= 0) return -1;
    if (!(m->n_amb > 0.0)) return -1;
    if (m->kind == ORC_GRID) {
        if (!m->grid || m->nx < 2 || m->ny < 2 || m->nz < 2) return -1;
    } else if (m->kind < 0 || m->kind > ORC_ZERNIKE || !m->params) {
        return -1;
    } else if (m->kind == ORC_SPHERICAL && m->n_params != 7) {
        return -1;
    } else if (m->kind == ORC_ZERNIKE) {
        if (m->n_params < 5) return -1;
        int K = (int)m->params[4];
        if (K < 0 || m->n_params != 5 + 3 * K || !(m->params[2] > 0.0) || !(m->params[3] > 0.0))
            return -1;
        for (int k = 0; k < K; ++k) {
            int j = (int)m->params[5 + 3 * k], l = (int)m->params[6 + 3 * k];
            if (j < 1 || j > 16 || l < 0 || l > 3) return -1;
        }
    } else if (m->kind == ORC_N2P &&
               (m->n_params != 4 || !(m->params[0] > 0.0) || !(m->params[1] > 0.0))) {
        return -1;
    }
    if (m->bkind < ORC_BOX || m->bkind > ORC_CYLINDER) return -1;
    return 0;
}

int orc_trace(const orc_medium *m, const orc_params *q, int64_t n, const double *P0,
              const double *d0, double *out_P, double *out_D, uint32_t *status,
              uint32_t *steps, uint32_t *ntir, uint32_t *nbtir, uint32_t *flags,
              int n_threads) {
    if (check_medium(m, q) || n < 0) return -1;
    if (n > 0 && (!P0 || !d0 || !out_P || !out_D || !status || !steps || !ntir || !nbtir ||
                  !flags))
        return -1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads > 0 ? n_threads : omp_get_max_threads())
    for (int64_t r = 0; r < n; ++r) {
        ray_out o;
        trace_one(m, q, P0 + 3 * r, d0 + 3 * r, &o, NULL);
        memcpy(out_P + 3 * r, o.P, sizeof o.P);
        memcpy(out_D + 3 * r, o.D, sizeof o.D);
        status[r] = o.status;
        steps[r] = o.steps;
        ntir[r] = o.ntir;
        nbtir[r] = o.nbtir;
        flags[r] = o.flags;
    }
    return 0;
}

int orc_trace_path(const orc_medium *m, const orc_params *q, const double *P0, const double *d0,
                   double *path, int64_t cap, int64_t *n_path, double *out_P, double *out_D,
                   uint32_t *status, uint32_t *steps, uint32_t *ntir, uint32_t *nbtir,
                   uint32_t *flags) {
    if (check_medium(m, q) || !P0 || !d0 || !n_path) return -1;
    path_rec pr = {path, path ? cap : 0, 0};
    ray_out o;
    trace_one(m, q, P0, d0, &o, &pr);
    *n_path = pr.n;
    if (out_P) memcpy(out_P, o.P, sizeof o.P);
    if (out_D) memcpy(out_D, o.D, sizeof o.D);
    if (status) *status = o.status;
    if (steps) *steps = o.steps;
    if (ntir) *ntir = o.ntir;
    if (nbtir) *nbtir = o.nbtir;
    if (flags) *flags = o.flags;
    return 0;
}

int orc_eval(const orc_medium *m, int64_t n, const double *P, double *n_out, double *g_out) {
    if (!m || n < 0 || (n > 0 && (!P || !n_out || !g_out))) return -1;
    for (int64_t r = 0; r < n; ++r) medium_eval(m, P + 3 * r, n_out + r, g_out + 3 * r);
    return 0;
}
