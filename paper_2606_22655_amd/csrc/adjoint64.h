// adjoint64.h -- reverse mode of the plain double-precision march through a
// discretized medium: the gradient of an exit-plane loss with respect to the
// grid's node values.
//
// One ray is a sequence of operations, each a function of a small state:
//   entry   launch -> first point on the surface, refracted direction
//           (case (i) with mu = n_amb / n(P_B));
//   decide  at P_i: n, grad n (trilinear, media.h), N = grad n / |grad n|
//           (Eq. (5)), then straight (cases (ii)/(iii)), TIR (Eqs. (19)-(20))
//           or vectorial Snell (Eqs. (9)-(10)), and the step Delta_i (Eq. (4));
//   move    P_{i+1} = P_i + Delta_i R_i (Eq. (3)) when the step stays inside;
//   btir    the step meets the surface and is reflected back (case (i));
//   exit    the step meets the surface, is refracted out and continues
//           straight to the exit plane, where the loss is taken.
// The operations are the same code, in the same order, as the forward march
// (lane64.h), so replaying them from a saved state reproduces its doubles
// bit for bit.  Each has a hand-written vector-Jacobian product (VJP): given
// the adjoint of the state after the operation it returns the adjoint of the
// state before it and adds the operation's contribution to the gradient of
// the node values (through n and grad n of the cell it evaluates).
//
// The derivative is that of the discrete march with its branch pattern held
// fixed (which decisions were Snell, TIR, straight, how many steps, where the
// surface was met): the march is piecewise smooth in the node values, and
// this is its gradient wherever no decision flips.
#pragma once

#include "lane64.h"

namespace vrt {
namespace adj {

enum { PH_DECIDE = 0, PH_MOVE = 1, PH_DONE = 2 };
enum { END_RUNNING = 0, END_PLANE = 1, END_OTHER = 2 };

struct St {  // state between operations
    d3 P, I, R;
    double n_last, Delta;
    uint32_t steps;
    int32_t phase;
};

struct Adj {  // adjoint of a state
    d3 P, I, R;
    double n_last, Delta;
};

__device__ __forceinline__ d3 zero3() { return mk(0.0, 0.0, 0.0); }
__device__ __forceinline__ Adj zero_adj() {
    Adj a;
    a.P = a.I = a.R = zero3();
    a.n_last = a.Delta = 0.0;
    return a;
}

// Gradient accumulation: node values (gv) and node central differences
// (gH, three arrays of nodes) of the cell that an evaluation touched.
struct GradOut {
    double *gv;
    double *gH;  // [3][nodes]
    size_t nodes;
};

__device__ __forceinline__ void grad_add(double *p, double v) {
#if defined(__HIP_DEVICE_COMPILE__)
    unsafeAtomicAdd(p, v);
#else
    *p += v;
#endif
}

// Per-lane accumulator of the node-gradient contributions of one cell: the
// 8 corners x (v, H_x, H_y, H_z) of the cell the lane last evaluated in.
// Consecutive steps of a ray mostly stay in one cell (a cell edge spans tens
// of steps), so contributions are summed here and added to the node arrays
// (atomically) only when the ray moves to another cell, and once at the end.
struct GradAcc {
    double *slot;     // 32 accumulators, `stride` apart
    uint32_t stride;
    int cell[3];      // cell held (cell[0] < 0: none)
    GradOut go;
    size_t nx, ny;

    __device__ void flush() {
        if (cell[0] < 0) return;
        for (int corner = 0; corner < 8; ++corner) {
            const int i = cell[0] + (corner & 1), j = cell[1] + ((corner >> 1) & 1),
                      k = cell[2] + (corner >> 2);
            const size_t node = ((size_t)k * ny + j) * nx + i;
            double *q = slot + (size_t)(4 * corner) * stride;
            if (q[0] != 0.0) grad_add(go.gv + node, q[0]);
            if (q[stride] != 0.0) grad_add(go.gH + node, q[stride]);
            if (q[2 * stride] != 0.0) grad_add(go.gH + go.nodes + node, q[2 * stride]);
            if (q[3 * stride] != 0.0) grad_add(go.gH + 2 * go.nodes + node, q[3 * stride]);
        }
        cell[0] = -1;
    }
    __device__ void open(const int c[3]) {
        if (cell[0] == c[0] && cell[1] == c[1] && cell[2] == c[2]) return;
        flush();
        for (int q = 0; q < 32; ++q) slot[(size_t)q * stride] = 0.0;
        cell[0] = c[0];
        cell[1] = c[1];
        cell[2] = c[2];
    }
};

__device__ inline GradAcc make_acc(double *slot, uint32_t stride, const MediumDev &m,
                                   const GradOut &go) {
    GradAcc a;
    a.slot = slot;
    a.stride = stride;
    a.cell[0] = a.cell[1] = a.cell[2] = -1;
    a.go = go;
    a.nx = (size_t)m.nx;
    a.ny = (size_t)m.ny;
    return a;
}

// VJP of the grid evaluation at P (media.h, med64<GRID>): n = sum_k w_k v_k and
// g_a = sum_k w_k H_a(k) over the 8 corners, w_k = prod_b (d_b ? f_b : 1 - f_b),
// f_b = (x_b - lo_b) / h_b - c_b.  Adds to the node gradients and returns the
// adjoint of P.
__device__ inline d3 grid_vjp(const MediumDev &m, d3 P, double nbar, d3 gbar, GradAcc &go) {
    const int nn[3] = {m.nx, m.ny, m.nz};
    int c[3];
    double f[3];
    bool inside[3];
    for (int a = 0; a < 3; ++a) {
        double x = get(P, a);
        inside[a] = !(x < m.lo[a]) && !(x > m.hi[a]);
        x = x < m.lo[a] ? m.lo[a] : (x > m.hi[a] ? m.hi[a] : x);
        const double u = (x - m.lo[a]) / m.h[a];
        int ci = (int)floor(u);
        ci = ci < 0 ? 0 : (ci > nn[a] - 2 ? nn[a] - 2 : ci);
        c[a] = ci;
        f[a] = u - (double)ci;
    }
    double fbar[3] = {0.0, 0.0, 0.0};
    go.open(c);
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const double wx = dx ? f[0] : 1.0 - f[0];
                const double wy = dy ? f[1] : 1.0 - f[1];
                const double wz = dz ? f[2] : 1.0 - f[2];
                const double w = wx * wy * wz;
                const int i = c[0] + dx, j = c[1] + dy, k = c[2] + dz;
                double v, hx, hy, hz;
                if (m.rec_exact) {  // the same doubles from the exact node record (media.h)
                    const float4 r = m.rec[((size_t)k * m.ny + j) * m.nx + i];
                    v = (double)r.x;
                    hx = (double)r.y / m.h[0];
                    hy = (double)r.z / m.h[1];
                    hz = (double)r.w / m.h[2];
                } else {
                    v = grid_node64(m, i, j, k);
                    hx = grid_cdiff64(m, i, j, k, 0);
                    hy = grid_cdiff64(m, i, j, k, 1);
                    hz = grid_cdiff64(m, i, j, k, 2);
                }
                const double sv = nbar * v + gbar.x * hx + gbar.y * hy + gbar.z * hz;
                fbar[0] += (dx ? 1.0 : -1.0) * wy * wz * sv;
                fbar[1] += (dy ? 1.0 : -1.0) * wx * wz * sv;
                fbar[2] += (dz ? 1.0 : -1.0) * wx * wy * sv;
                double *q = go.slot + (size_t)(4 * (dz * 4 + dy * 2 + dx)) * go.stride;
                q[0] += w * nbar;
                q[go.stride] += w * gbar.x;
                q[2 * go.stride] += w * gbar.y;
                q[3 * go.stride] += w * gbar.z;
            }
    return mk(inside[0] ? fbar[0] / m.h[0] : 0.0, inside[1] ? fbar[1] / m.h[1] : 0.0,
              inside[2] ? fbar[2] / m.h[2] : 0.0);
}

// VJP of snell64 (R = mu I + gamma N, gamma = -mu c + sgn(c) sqrt(D),
// c = N.I passed in, D = 1 - mu^2 (1 - c^2)) given Rbar: adds to Ibar, Nbar and
// returns mubar; c's dependence on N and I is included.
__device__ inline double snell_vjp(d3 I, d3 N, double mu, double c, double D, d3 Rbar, d3 &Ibar,
                                   d3 &Nbar) {
    const double sg = c > 0.0 ? 1.0 : -1.0;
    const double sD = sqrt(D);
    const double gam = -mu * c + sg * sD;
    Ibar = Ibar + mu * Rbar;
    Nbar = Nbar + gam * Rbar;
    double mubar = dot(I, Rbar);
    const double gbar = dot(N, Rbar);
    mubar += -c * gbar;
    double cbar = -mu * gbar;
    const double Dbar = sg * gbar / (2.0 * sD);
    mubar += Dbar * (-2.0 * mu * (1.0 - c * c));
    cbar += Dbar * (2.0 * mu * mu * c);
    Nbar = Nbar + cbar * I;
    Ibar = Ibar + cbar * N;
    return mubar;
}

// VJP of reflect64 (R = v / |v|, v = I - 2 c N, c = N.I passed in).
__device__ inline void reflect_vjp(d3 I, d3 N, double c, d3 Rbar, d3 &Ibar, d3 &Nbar) {
    const d3 v = I - (2.0 * c) * N;
    const double l = sqrt(dot(v, v));
    const d3 R = mk(v.x / l, v.y / l, v.z / l);
    const d3 vbar = (1.0 / l) * (Rbar - dot(R, Rbar) * R);
    Ibar = Ibar + vbar;
    const double cbar = -2.0 * dot(N, vbar);
    Nbar = Nbar + (-2.0 * c) * vbar;
    Nbar = Nbar + cbar * I;
    Ibar = Ibar + cbar * N;
}

// Entry from a launch state (as lane64.h).  Returns the state after entry.
__device__ inline void fwd_entry(const MediumDev &m, const BoundaryDev &b, const TraceDev &t, d3 P0,
                                 d3 d0, St &s, int &end) {
    s.steps = 0;
    s.Delta = 0.0;
    end = END_RUNNING;
    const double l0 = sqrt(dot(d0, d0));
    if (!isfinite(P0.x) || !isfinite(P0.y) || !isfinite(P0.z) || !isfinite(l0) || !(l0 > 0.0)) {
        end = END_OTHER;
        s.phase = PH_DONE;
        return;
    }
    s.I = mk(d0.x / l0, d0.y / l0, d0.z / l0);
    s.P = P0;
    s.R = s.I;
    if (surf_inside_strict(b, s.P)) {
        s.n_last = index64<VRT_MEDIUM_GRID>(m, s.P);
        s.phase = PH_DECIDE;
        return;
    }
    double tt;
    int face;
    if (!surf_entry(b, s.P, s.I, tt, face)) {
        end = END_OTHER;
        s.phase = PH_DONE;
        return;
    }
    s.P = s.P + tt * s.I;
    surf_snap(b, s.P, face);
    const d3 N = surf_normal(b, s.P, face);
    const double n_in = index64<VRT_MEDIUM_GRID>(m, s.P);
    const double mu = m.n_amb / n_in, c = dot(N, s.I);
    const double D = 1.0 - mu * mu * (1.0 - c * c);
    if (D <= 0.0) {
        end = END_OTHER;
        s.phase = PH_DONE;
        return;
    }
    s.R = snell64(s.I, N, mu, c, D);
    s.n_last = n_in;
    s.Delta = t.dL0 / n_in;
    s.phase = PH_MOVE;
}

// One operation (decide, or a move that may meet the surface).  At the exit
// the point on the exit plane is returned in (x, y).
__device__ inline void fwd_op(const MediumDev &m, const BoundaryDev &b, const TraceDev &t, St &s,
                              double &x, double &y, int &end) {
    if (s.phase == PH_DECIDE) {
        double ni;
        d3 g;
        med64<VRT_MEDIUM_GRID>(m, s.P, ni, g);
        const double gl = sqrt(dot(g, g));
        if (!isfinite(gl) || gl == 0.0) {
            s.R = s.I;
            s.Delta = t.dL0 / ni;
        } else {
            const d3 N = mk(g.x / gl, g.y / gl, g.z / gl);
            const double c = dot(N, s.I);
            if (fabs(c) <= t.eps_tan) {  // case (iv), Eqs. (16)-(18)
                s.Delta = t.dL0 / ni;
                const double dn = index64<VRT_MEDIUM_GRID>(m, s.P + s.Delta * N) - ni;
                const double a = dn / (2.0 * ni);
                const double w = 1.0 - a * a;
                const d3 v = sqrt(w > 0.0 ? w : 0.0) * s.I + a * N;
                const double lv = sqrt(dot(v, v));
                s.R = mk(v.x / lv, v.y / lv, v.z / lv);
            } else {
                const double mu = s.n_last / ni;
                const double D = 1.0 - mu * mu * (1.0 - c * c);
                if (D <= 0.0) {
                    s.R = reflect64(s.I, N, c);
                    s.Delta = t.dL0 / s.n_last;
                } else {
                    s.R = snell64(s.I, N, mu, c, D);
                    s.Delta = t.dL0 / ni;
                }
            }
        }
        s.n_last = ni;
        s.phase = PH_MOVE;
        return;
    }
    int face;
    const double tx = surf_exit(b, s.P, s.R, face);
    s.steps++;
    if (tx > s.Delta) {
        s.P = s.P + s.Delta * s.R;
        s.I = s.R;
        s.phase = PH_DECIDE;
        if ((int64_t)s.steps >= t.max_steps) {
            s.phase = PH_DONE;
            end = END_OTHER;
        }
        return;
    }
    d3 Pb = s.P + tx * s.R;
    surf_snap(b, Pb, face);
    const d3 N = surf_normal(b, Pb, face);
    const double mu = s.n_last / m.n_amb, c = dot(N, s.R);
    const double D = 1.0 - mu * mu * (1.0 - c * c);
    if (D <= 0.0) {
        s.R = reflect64(s.R, N, c);
        s.Delta = t.dL0 / s.n_last;
        s.n_last = index64<VRT_MEDIUM_GRID>(m, Pb);
        s.P = Pb;
        if ((int64_t)s.steps >= t.max_steps) {
            s.phase = PH_DONE;
            end = END_OTHER;
        }
        return;
    }
    const d3 Ro = snell64(s.R, N, mu, c, D);
    s.phase = PH_DONE;
    if (!(Ro.z > 0.0) || (t.plane_z - Pb.z) / Ro.z < 0.0) {
        end = END_OTHER;
        return;
    }
    const double sp = (t.plane_z - Pb.z) / Ro.z;
    x = Pb.x + sp * Ro.x;
    y = Pb.y + sp * Ro.y;
    end = END_PLANE;
}

// VJP of Pb = snap(P + tx R) with tx = surf_exit (box face `face`): the face
// coordinate is fixed; the others move with P and R; tx moves with P and R
// through (face - P_k) / R_k.
__device__ inline void surface_point_vjp(const BoundaryDev &b, d3 P, d3 R, double tx, int face,
                                         d3 Pbbar, d3 &Pbar, d3 &Rbar) {
    const int k = face % 3;
    double txbar = 0.0;
    for (int j = 0; j < 3; ++j) {
        if (j == k) continue;
        set(Pbar, j, get(Pbar, j) + get(Pbbar, j));
        set(Rbar, j, get(Rbar, j) + tx * get(Pbbar, j));
        txbar += get(R, j) * get(Pbbar, j);
    }
    const double rk = get(R, k);
    if (tx > 0.0 && rk != 0.0) {
        set(Pbar, k, get(Pbar, k) - txbar / rk);
        set(Rbar, k, get(Rbar, k) - txbar * tx / rk);
    }
}

// VJP of one operation from its input state s.  a: adjoint of the state after
// the operation on entry, of the state before it on return.  (xbar, ybar):
// adjoint of the exit-plane point, used when the operation is the exit.
__device__ inline void vjp_op(const MediumDev &m, const BoundaryDev &b, const TraceDev &t,
                              const St &s, Adj &a, double xbar, double ybar, GradAcc &go) {
    if (s.phase == PH_DECIDE) {
        double ni;
        d3 g;
        med64<VRT_MEDIUM_GRID>(m, s.P, ni, g);
        const double gl = sqrt(dot(g, g));
        d3 Ibar = a.I, gbar = zero3();
        double nibar = a.n_last, nlbar = 0.0;
        if (!isfinite(gl) || gl == 0.0) {  // R = I, Delta = dL0 / ni
            Ibar = Ibar + a.R;
            nibar += -a.Delta * t.dL0 / (ni * ni);
        } else {
            const d3 N = mk(g.x / gl, g.y / gl, g.z / gl);
            const double c = dot(N, s.I);
            const double mu = s.n_last / ni;
            const double D = 1.0 - mu * mu * (1.0 - c * c);
            d3 Nbar = zero3();
            if (fabs(c) <= t.eps_tan) {
                // exact tangency (a set of measure zero): R = I to first order in
                // the probe's index difference; only that term is carried
                Ibar = Ibar + a.R;
                nibar += -a.Delta * t.dL0 / (ni * ni);
            } else if (D <= 0.0) {
                reflect_vjp(s.I, N, c, a.R, Ibar, Nbar);
                nlbar += -a.Delta * t.dL0 / (s.n_last * s.n_last);
            } else {
                const double mubar = snell_vjp(s.I, N, mu, c, D, a.R, Ibar, Nbar);
                nlbar += mubar / ni;
                nibar += -mubar * s.n_last / (ni * ni);
                nibar += -a.Delta * t.dL0 / (ni * ni);
            }
            gbar = (1.0 / gl) * (Nbar - dot(N, Nbar) * N);
        }
        const d3 Pg = grid_vjp(m, s.P, nibar, gbar, go);
        a.P = a.P + Pg;
        a.I = Ibar;
        a.R = zero3();
        a.n_last = nlbar;
        a.Delta = 0.0;
        return;
    }
    int face;
    const double tx = surf_exit(b, s.P, s.R, face);
    if (tx > s.Delta) {  // move
        const d3 Pbar = a.P;
        a.R = a.R + a.I + s.Delta * Pbar;
        a.Delta = a.Delta + dot(s.R, Pbar);
        a.I = zero3();
        return;
    }
    d3 Pb = s.P + tx * s.R;
    surf_snap(b, Pb, face);
    const d3 N = surf_normal(b, Pb, face);
    const double mu = s.n_last / m.n_amb, c = dot(N, s.R);
    const double D = 1.0 - mu * mu * (1.0 - c * c);
    d3 Pbbar = zero3(), Pbar = zero3(), Rbar = zero3(), Nbar = zero3();
    double nlbar = 0.0;
    if (D <= 0.0) {  // boundary TIR: P' = Pb, R' = reflect, Delta' = dL0/n_last, n' = n(Pb)
        Pbbar = a.P + grid_vjp(m, Pb, a.n_last, zero3(), go);
        reflect_vjp(s.R, N, c, a.R, Rbar, Nbar);
        nlbar = -a.Delta * t.dL0 / (s.n_last * s.n_last);
        surface_point_vjp(b, s.P, s.R, tx, face, Pbbar, Pbar, Rbar);
        a.P = Pbar;
        a.R = Rbar;
        a.n_last = nlbar;
        a.Delta = 0.0;
        // I passes through
        return;
    }
    // exit: Ro = snell, then the straight line to the plane z = plane_z
    const d3 Ro = snell64(s.R, N, mu, c, D);
    const double sp = (t.plane_z - Pb.z) / Ro.z;
    d3 Robar = mk(sp * xbar, sp * ybar, 0.0);
    Pbbar = mk(xbar, ybar, 0.0);
    const double spbar = Ro.x * xbar + Ro.y * ybar;
    Pbbar.z += -spbar / Ro.z;
    Robar.z += -spbar * sp / Ro.z;
    const double mubar = snell_vjp(s.R, N, mu, c, D, Robar, Rbar, Nbar);
    nlbar = mubar / m.n_amb;
    surface_point_vjp(b, s.P, s.R, tx, face, Pbbar, Pbar, Rbar);
    a.P = Pbar;
    a.R = Rbar;
    a.I = zero3();
    a.n_last = nlbar;
    a.Delta = 0.0;
}

// VJP of the entry: the launch state is not differentiated, the node values
// are (through n at the entry point).
__device__ inline void vjp_entry(const MediumDev &m, const BoundaryDev &b, const TraceDev &t, d3 P0,
                                 d3 d0, const Adj &a, GradAcc &go) {
    const double l0 = sqrt(dot(d0, d0));
    const d3 I = mk(d0.x / l0, d0.y / l0, d0.z / l0);
    d3 P = P0;
    if (surf_inside_strict(b, P)) {
        grid_vjp(m, P, a.n_last, zero3(), go);
        return;
    }
    double tt;
    int face;
    if (!surf_entry(b, P, I, tt, face)) return;
    P = P + tt * I;
    surf_snap(b, P, face);
    const d3 N = surf_normal(b, P, face);
    const double n_in = index64<VRT_MEDIUM_GRID>(m, P);
    const double mu = m.n_amb / n_in, c = dot(N, I);
    const double D = 1.0 - mu * mu * (1.0 - c * c);
    d3 Ibar = zero3(), Nbar = zero3();
    const double mubar = snell_vjp(I, N, mu, c, D, a.R, Ibar, Nbar);
    const double nbar = -mubar * m.n_amb / (n_in * n_in) + a.n_last - a.Delta * t.dL0 / (n_in * n_in);
    grid_vjp(m, P, nbar, zero3(), go);
}

// Node central differences H_a(p) = (v[hi] - v[lo]) / span (media.h,
// grid_cdiff64) transposed: the adjoint of H_a at node p goes to v[hi] with
// +1/span and to v[lo] with -1/span.
__device__ inline void cdiff_transpose(const MediumDev &m, size_t p, const double *gH, double *gv,
                                       size_t nodes) {
    const int ii = (int)(p % (size_t)m.nx);
    const int jj = (int)((p / (size_t)m.nx) % (size_t)m.ny);
    const int kk = (int)(p / ((size_t)m.nx * m.ny));
    const int nn[3] = {m.nx, m.ny, m.nz};
    const int id[3] = {ii, jj, kk};
    const size_t stride[3] = {1, (size_t)m.nx, (size_t)m.nx * m.ny};
    for (int a = 0; a < 3; ++a) {
        const double hb = gH[(size_t)a * nodes + p];
        if (hb == 0.0) continue;
        int lo = id[a], hi = id[a];
        double span;
        if (id[a] == 0) {
            hi = 1;
            span = m.h[a];
        } else if (id[a] == nn[a] - 1) {
            lo = nn[a] - 2;
            span = m.h[a];
        } else {
            lo = id[a] - 1;
            hi = id[a] + 1;
            span = 2.0 * m.h[a];
        }
        const size_t base = p - (size_t)id[a] * stride[a];
        grad_add(gv + base + (size_t)hi * stride[a], hb / span);
        grad_add(gv + base + (size_t)lo * stride[a], -hb / span);
    }
}

}  // namespace adj
}  // namespace vrt
