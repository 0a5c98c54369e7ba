/*
 * vrt_oracle.h -- C interface of the plain FP64 CPU oracle for the
 * constant-optical-path-length vectorial ray march (VRT) in gradient-index
 * media.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header or
 * constant with the GPU library.
 *
 * All arrays are host memory, row-major (n, 3) for points and directions.
 */
#ifndef VRT_ORACLE_H
#define VRT_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* medium kinds */
enum {
    ORC_HOMOGENEOUS = 0, /* params [n_h]                                         */
    ORC_LINEAR = 1,      /* params [n0, gx, gy, gz]      n = n0 + g.P             */
    ORC_LUNEBURG = 2,    /* params [R, cx, cy, cz]       n = sqrt(2 - r^2/R^2)    */
    ORC_FIBER = 3,       /* params [n_c, Delta, R, cx, cy]  Sec. IV, Eq. (21)     */
    ORC_GAUSSIAN = 4,    /* params [n0, K, (A, sigma, cx, cy, cz) x K]            */
    ORC_GRID = 5,        /* trilinear grid, node-central-difference gradient      */
    ORC_SPHERICAL = 6,   /* params [a0, a1, a2, a3, cx, cy, cz]  Sec. V, Eq. (26) */
    ORC_N2P = 7,         /* params [R, F, beta, gamma]  Sec. VI, Eq. (27), axis z */
    ORC_ZERNIKE = 8      /* params [n_lo, n_hi, rho_max, z_max, K, (j, l, c) x K]
                          * Sec. V: Fringe Zernike j <= 16 times Legendre l <= 3 */
};

/* boundary kinds (convex enclosing surface, Sec. II case (i)) */
enum { ORC_BOX = 0, ORC_SPHERE = 1, ORC_CYLINDER = 2 };

/* per-ray status */
enum {
    ORC_EXITED = 0, ORC_MISSED = 1, ORC_TRUNCATED = 2, ORC_NO_PLANE = 3,
    ORC_INVALID_INPUT = 4, ORC_REFLECTED_AT_ENTRY = 5
};

/* per-ray flag bits */
enum {
    ORC_F_NEAR_CRITICAL = 1, ORC_F_TANGENT = 2, ORC_F_STRAIGHT = 4, ORC_F_BOUNDARY_TIR = 8,
    ORC_F_NEAR_TIE = 16,    /* a step ended within tie_eps (perpendicular) of the surface */
    ORC_F_NEAR_GRAZING = 32, /* a refraction into higher index had |N.I| < crit_rad */
    /* the same three windows ten times wider */
    ORC_F_NEAR_CRITICAL_WIDE = 64, ORC_F_NEAR_TIE_WIDE = 128, ORC_F_NEAR_GRAZING_WIDE = 256
};

typedef struct {
    int32_t kind;
    int32_t n_params;
    const double *params;
    const float *grid;     /* ORC_GRID: nz*ny*nx values, x fastest */
    int32_t nx, ny, nz;
    int32_t bkind;
    double glo[3], ghi[3]; /* ORC_GRID: positions of the first and last nodes */
    double bparams[6];     /* box [lo3, hi3]; sphere [c3, r]; cylinder [cx, cy, r, z0, z1] */
    double n_amb;          /* index of the homogeneous surroundings */
} orc_medium;

typedef struct {
    double dL0;          /* optical path length of every step, Eqs. (3)-(4) */
    int64_t max_steps;   /* guard for trapped rays -> ORC_TRUNCATED */
    double eps_tan;      /* |N.I| <= eps_tan selects the tangential rule (iv) */
    double crit_rad;     /* near-critical flag window in radians */
    double tie_eps;      /* near-tie flag window: distance of a step end from the surface */
    double plane_z;      /* exit plane z (used when has_plane != 0) */
    int32_t has_plane;
    int32_t pad;
} orc_params;

/* Trace n rays.  P0, d0: (n,3).  Outputs: exit point/direction (n,3), status,
 * steps, interior TIR count, boundary TIR count, flags (n each).
 * n_threads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad arguments. */
int orc_trace(const orc_medium *m, const orc_params *q, int64_t n,
              const double *P0, const double *d0,
              double *out_P, double *out_D, uint32_t *status, uint32_t *steps,
              uint32_t *ntir, uint32_t *nbtir, uint32_t *flags, int n_threads);

/* Trace one ray and record every point P_i it passes through (launch point,
 * entry point, every step end and every boundary point) into path (cap x 3).
 * *n_path receives the number of points produced (may exceed cap; only the
 * first cap are stored). */
int orc_trace_path(const orc_medium *m, const orc_params *q,
                   const double *P0, const double *d0, double *path, int64_t cap,
                   int64_t *n_path, double *out_P, double *out_D, uint32_t *status,
                   uint32_t *steps, uint32_t *ntir, uint32_t *nbtir, uint32_t *flags);

/* Evaluate n and grad n at n points P (n,3). */
int orc_eval(const orc_medium *m, int64_t n, const double *P, double *n_out, double *g_out);

#ifdef __cplusplus
}
#endif
#endif
