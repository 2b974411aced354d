/*
 * eik_oracle.c -- plain, slow, single-threaded FP64 reference for the
 * Randers-Finsler fast-sweeping eikonal solve and its implicit-differentiation
 * adjoint ("Differentiable Randers-Finsler Eikonal Solvers", arXiv 2603.00035).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's library. It shares no code, header,
 * table or helper with the HIP implementation; it is written from the paper.
 *
 * Conventions (Sec. 3.1-3.2, App. "Solver details", Fig. stencil):
 *   node (i,j), 0<=i<nx, 0<=j<ny, flat index j*nx+i, position (i*h, j*h);
 *   fields are row-major planes: M = [m11 | m12 | m22], omega = [bx | by];
 *   eight neighbours numbered counter-clockwise from the upper-left one
 *   (+y is +j); stencil k uses neighbours k and (k+1) mod 8;
 *   displacement of a donor, m, points from the donor to the receiving node,
 *   the reading under which the one-point update T0 = T_i + m.b + |m|_G solves
 *   the eikonal PDE (grad T - b)^T G^-1 (grad T - b) = 1 (Eq. randers_eikonal).
 *
 * Readings of the paper that this file takes (each is listed with its reason
 * in the design notes of the repository):
 *   - every finite neighbour contributes a one-point candidate (Sec. 3.2 text:
 *     "set T to the smallest valid candidate"), not only on two-point failure;
 *   - causality is tested against the candidate value (App. solver details);
 *   - the update overwrites T (no min with the previous value);
 *   - a full four-sweep cycle with no change above tol ends the solve;
 *   - ties between candidates keep the first in the order
 *     two-point k=0..7, then one-point k=0..7 (strict <).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Neighbour k sits at (i + NBX[k], j + NBY[k]). Counter-clockwise from upper-left. */
static const int NBX[8] = {-1, -1, -1, 0, 1, 1, 1, 0};
static const int NBY[8] = {1, 0, -1, -1, -1, 0, 1, 1};

enum { ORA_SOURCE = 0xFE, ORA_UNREACHED = 0xFF };

/* ------------------------------------------------------------------------- */
/* Local solves (Eq. two_point, Eq. one_point; App. solver details).           */
/* ------------------------------------------------------------------------- */

/* G = [[g11,g12],[g12,g22]] applied as a quadratic form u^T G v. */
static double gform(const double g[3], double ux, double uy, double vx, double vy)
{
    return g[0] * ux * vx + g[1] * (ux * vy + uy * vx) + g[2] * uy * vy;
}

/* One-point update, Eq. one_point: T0 = T_k + m.b + sqrt(m^T G m), with the
 * physical displacement m = h * (receiver - donor). */
static double one_point(const double g[3], const double b[2], double h, int k, double Tk)
{
    double mx = -h * NBX[k], my = -h * NBY[k];
    return Tk + (mx * b[0] + my * b[1]) + sqrt(gform(g, mx, my, mx, my));
}

/* Two-point (triangular) update, Eq. two_point. Donors are neighbours kp, kq
 * with times Tp, Tq. Returns 1 and the candidate when it is valid:
 *   E = Mst^T G Mst, Q = E^-1, S_a = T_a + m_a.b,
 *   T0 = larger root of (S - T0 1)^T Q (S - T0 1) = 1,
 *   valid iff lambda = Q (T0 1 - S) >= 0 (geometric validity) and T0 > T_a
 *   for both donors (causality).
 * The quadratic is written for tau = T0 - S0 with S0 = min(S1, S2); this is an
 * exact change of variable that keeps all terms of one scale. lam[] receives
 * the barycentric coordinates and Qu[] the vector Q u with u = S - T0 1. */
static int two_point(const double g[3], const double b[2], double h, int kp, int kq,
                     double Tp, double Tq, double *T0_out, double lam[2], double Qu[2])
{
    double m1x = -h * NBX[kp], m1y = -h * NBY[kp];
    double m2x = -h * NBX[kq], m2y = -h * NBY[kq];
    double E11 = gform(g, m1x, m1y, m1x, m1y);
    double E12 = gform(g, m1x, m1y, m2x, m2y);
    double E22 = gform(g, m2x, m2y, m2x, m2y);
    double det = E11 * E22 - E12 * E12;
    double Q11 = E22 / det, Q12 = -E12 / det, Q22 = E11 / det;
    double S1 = Tp + (m1x * b[0] + m1y * b[1]);
    double S2 = Tq + (m2x * b[0] + m2y * b[1]);
    double S0 = S1 < S2 ? S1 : S2;
    double s1 = S1 - S0, s2 = S2 - S0;
    /* (s - tau 1)^T Q (s - tau 1) = 1  <=>  A tau^2 - 2 B tau + C = 0 */
    double A = Q11 + 2.0 * Q12 + Q22;
    double B = Q11 * s1 + Q12 * (s1 + s2) + Q22 * s2;
    double C = Q11 * s1 * s1 + 2.0 * Q12 * s1 * s2 + Q22 * s2 * s2 - 1.0;
    double D = B * B - A * C;
    if (!(D >= 0.0)) return 0;
    double tau = (B + sqrt(D)) / A; /* larger root */
    double T0 = S0 + tau;
    double l1 = Q11 * (tau - s1) + Q12 * (tau - s2);
    double l2 = Q12 * (tau - s1) + Q22 * (tau - s2);
    if (lam) { lam[0] = l1; lam[1] = l2; }
    if (Qu) { Qu[0] = -l1; Qu[1] = -l2; } /* Q u = Q (S - T0 1) = -lambda */
    *T0_out = T0;
    return (l1 >= 0.0 && l2 >= 0.0 && T0 > Tp && T0 > Tq) ? 1 : 0;
}

typedef struct {
    int nx, ny;
    double h;
    const double *M, *om;
} ora_field;

static void params_at(const ora_field *f, int c, double g[3], double b[2])
{
    size_t n = (size_t)f->nx * f->ny;
    g[0] = f->M[c];
    g[1] = f->M[n + c];
    g[2] = f->M[2 * n + c];
    b[0] = f->om[c];
    b[1] = f->om[n + c];
}

/* Neighbour times of node (i,j); +inf outside the grid (free outflow edge). */
static void neighbour_times(const ora_field *f, const double *T, int i, int j, double Tn[8])
{
    for (int k = 0; k < 8; ++k) {
        int a = i + NBX[k], bb = j + NBY[k];
        Tn[k] = (a < 0 || a >= f->nx || bb < 0 || bb >= f->ny) ? INFINITY : T[(size_t)bb * f->nx + a];
    }
}

/* Minimum over the valid candidates at one node (Sec. 3.2, Alg. forward).
 * code receives the winner: 0..7 two-point stencil, 8..15 one-point, 0xFF none. */
static double local_update(const ora_field *f, const double *T, int i, int j, int one_point_only, int *code)
{
    double g[3], b[2], Tn[8];
    int c = j * f->nx + i;
    params_at(f, c, g, b);
    neighbour_times(f, T, i, j, Tn);
    double best = INFINITY;
    int win = ORA_UNREACHED;
    if (!one_point_only) {
        for (int k = 0; k < 8; ++k) {
            int kq = (k + 1) & 7;
            if (!isfinite(Tn[k]) || !isfinite(Tn[kq])) continue;
            double t;
            if (two_point(g, b, f->h, k, kq, Tn[k], Tn[kq], &t, NULL, NULL) && t < best) {
                best = t;
                win = k;
            }
        }
    }
    for (int k = 0; k < 8; ++k) {
        if (!isfinite(Tn[k])) continue;
        double t = one_point(g, b, f->h, k, Tn[k]);
        if (t < best) {
            best = t;
            win = 8 + k;
        }
    }
    if (code) *code = win;
    return best;
}

/* ------------------------------------------------------------------------- */
/* Forward solve (Alg. forward; Sec. 3.2).                                    */
/* ------------------------------------------------------------------------- */

/* Whether a change from a to b counts toward non-convergence: |b-a| > tol*|b|,
 * and any change between infinite and finite. tol = 0 means exact stationarity. */
static int counts_as_change(double a, double b, double tol)
{
    if (a == b) return 0;
    if (!isfinite(a) || !isfinite(b)) return 1;
    return fabs(b - a) > tol * fabs(b);
}

/* mode 0: Gauss-Seidel raster sweeps in the four orderings (i+,j+), (i-,j+),
 *         (i-,j-), (i+,j-), cycled; converged after a cycle with no change.
 * mode 1: Jacobi iteration (every node from the previous iterate; App.
 *         comparisons, the Jacobi baseline); converged after one iteration
 *         with no change.
 * mode 2: the Gauss-Seidel sweeps of mode 0 with every stored value rounded
 *         to the nearest single-precision number (each update is still
 *         evaluated exactly in double precision): the fixed point a solve
 *         that stores T in single precision can reach at best. Used only to
 *         measure that storage's effect on the adjoint, never as a parity
 *         reference.
 * T_init (optional) replaces the +inf initialisation; the update overwrites.
 * Returns 0 when converged, 1 when max_sweeps was reached. */
int ora_forward(int nx, int ny, double h, const double *M, const double *om, int n_src,
                const int *src_idx, const double *src_t, const double *T_init, int mode,
                int one_point_only, int max_sweeps, double tol, double *T, int *sweeps_out)
{
    ora_field f = {nx, ny, h, M, om};
    size_t n = (size_t)nx * ny;
    unsigned char *is_src = (unsigned char *)calloc(n, 1);
    double *Told = mode == 1 ? (double *)malloc(n * sizeof(double)) : NULL;
    for (size_t c = 0; c < n; ++c) T[c] = T_init ? T_init[c] : INFINITY;
    for (int s = 0; s < n_src; ++s) {
        is_src[src_idx[s]] = 1;
        T[src_idx[s]] = src_t ? src_t[s] : 0.0;
    }
    int sweeps = 0, quiet = 0, status = 1;
    while (sweeps < max_sweeps) {
        int changed = 0;
        if (mode == 1) {
            memcpy(Told, T, n * sizeof(double));
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t c = (size_t)j * nx + i;
                    if (is_src[c]) continue;
                    double t = local_update(&f, Told, i, j, one_point_only, NULL);
                    changed |= counts_as_change(Told[c], t, tol);
                    T[c] = t;
                }
            ++sweeps;
            if (!changed) { status = 0; break; }
            continue;
        }
        int dir = sweeps & 3;
        int ifwd = (dir == 0 || dir == 3), jfwd = (dir == 0 || dir == 1);
        for (int jj = 0; jj < ny; ++jj) {
            int j = jfwd ? jj : ny - 1 - jj;
            for (int ii = 0; ii < nx; ++ii) {
                int i = ifwd ? ii : nx - 1 - ii;
                size_t c = (size_t)j * nx + i;
                if (is_src[c]) continue;
                double t = local_update(&f, T, i, j, one_point_only, NULL);
                if (mode == 2) t = (double)(float)t;
                changed |= counts_as_change(T[c], t, tol);
                T[c] = t;
            }
        }
        ++sweeps;
        quiet = changed ? 0 : quiet + 1;
        if (quiet >= 4) { status = 0; break; }
    }
    if (sweeps_out) *sweeps_out = sweeps;
    free(is_src);
    free(Told);
    return status;
}

/* One evaluation of the local update at node c from the field T, for tests:
 * returns the minimum candidate and its code. */
double ora_local_update(int nx, int ny, double h, const double *M, const double *om,
                        const double *T, int c, int one_point_only, int *code)
{
    ora_field f = {nx, ny, h, M, om};
    return local_update(&f, T, c % nx, c / nx, one_point_only, code);
}

/* The local update evaluated at every node of the field T (no node is
 * changed), for tests that check whether a field is a fixed point of the
 * update: out_v[c] and out_code[c] are the minimum candidate and its code. */
void ora_local_update_all(int nx, int ny, double h, const double *M, const double *om, const double *T,
                          double *out_v, unsigned char *out_code)
{
    ora_field f = {nx, ny, h, M, om};
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int code;
            out_v[(size_t)j * nx + i] = local_update(&f, T, i, j, 0, &code);
            out_code[(size_t)j * nx + i] = (unsigned char)code;
        }
}

/* Two-point solve exposed for tests: returns validity, candidate, lambda. */
int ora_two_point(const double g[3], const double b[2], double h, int kp, int kq,
                  double Tp, double Tq, double *T0, double lam[2])
{
    return two_point(g, b, h, kp, kq, Tp, Tq, T0, lam, NULL);
}

double ora_one_point(const double g[3], const double b[2], double h, int k, double Tk)
{
    return one_point(g, b, h, k, Tk);
}

/* ------------------------------------------------------------------------- */
/* Active stencils and dependency levels (Alg. backward, stencil identification) */
/* ------------------------------------------------------------------------- */

static int cmp_dec_T_values;
static const double *cmp_T;
static int cmp_order(const void *a, const void *b)
{
    int ia = *(const int *)a, ib = *(const int *)b;
    double ta = cmp_T[ia], tb = cmp_T[ib];
    if (ta != tb) return cmp_dec_T_values ? (ta < tb ? 1 : -1) : (ta < tb ? -1 : 1);
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

/* Reached nodes sorted by T (decreasing if dec, else increasing), ties by index. */
static int *sorted_reached(const double *T, size_t n, int dec, size_t *count)
{
    int *ord = (int *)malloc(n * sizeof(int));
    size_t m = 0;
    for (size_t c = 0; c < n; ++c)
        if (isfinite(T[c])) ord[m++] = (int)c;
    cmp_T = T;
    cmp_dec_T_values = dec;
    qsort(ord, m, sizeof(int), cmp_order);
    *count = m;
    return ord;
}

/* Donors of a winner code at node (i,j): returns their count (0, 1 or 2). */
static int donors_of(int code, int i, int j, int nx, int d[2], int dk[2])
{
    if (code < 8) {
        dk[0] = code;
        dk[1] = (code + 1) & 7;
        d[0] = (j + NBY[dk[0]]) * nx + (i + NBX[dk[0]]);
        d[1] = (j + NBY[dk[1]]) * nx + (i + NBX[dk[1]]);
        return 2;
    }
    if (code < 16) {
        dk[0] = code - 8;
        d[0] = (j + NBY[dk[0]]) * nx + (i + NBX[dk[0]]);
        return 1;
    }
    return 0;
}

/* Winner code per node from the final field (sources 0xFE, unreached 0xFF),
 * and the dependency level: 0 at sources, 1 + max over the donors otherwise,
 * computed in increasing-T order (donors have strictly smaller T). */
void ora_parents_levels(int nx, int ny, double h, const double *M, const double *om, int n_src,
                        const int *src_idx, const double *T, unsigned char *parent, int *level)
{
    ora_field f = {nx, ny, h, M, om};
    size_t n = (size_t)nx * ny;
    for (size_t c = 0; c < n; ++c) {
        int code = ORA_UNREACHED;
        if (isfinite(T[c])) local_update(&f, T, (int)(c % nx), (int)(c / nx), 0, &code);
        parent[c] = (unsigned char)code;
        level[c] = -1;
    }
    for (int s = 0; s < n_src; ++s) parent[src_idx[s]] = ORA_SOURCE;
    size_t m;
    int *ord = sorted_reached(T, n, 0, &m);
    for (size_t q = 0; q < m; ++q) {
        int c = ord[q];
        if (parent[c] == ORA_SOURCE) { level[c] = 0; continue; }
        int d[2], dk[2];
        int nd = donors_of(parent[c], c % nx, c / nx, nx, d, dk);
        int lv = -1;
        for (int a = 0; a < nd; ++a)
            if (level[d[a]] > lv) lv = level[d[a]];
        level[c] = nd ? lv + 1 : -1;
    }
    free(ord);
}

/* ------------------------------------------------------------------------- */
/* Residual Jacobian and partials (Eq. jacobian_planar, Eq. two_point_partials,  */
/* Eq. one_point_partials).                                                    */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nd;          /* number of donors */
    int d[2];        /* donor node indices */
    double Jii;      /* dR_i/dT_i */
    double Jid[2];   /* dR_i/dT_donor */
    double dRdb[2];  /* dR_i/db */
    double dRdG[3];  /* dR_i/dG as (G11, G12, G22) of the symmetric 2x2 matrix */
} ora_row;

/* Residual row of node c for its active update, evaluated at the converged T.
 * Two-point: R = u^T Q u - 1, u = S - T0 1:
 *   dR/dT0 = -2 1^T Q u, dR/dT_k = 2 e_k^T Q u,
 *   dR/db = 2 Mst Q u, dR/dG = -Mst Q u u^T Q Mst^T.
 * One-point: r = T_k + m.b - T0, e = m^T G m, R = r^2 - e:
 *   dR/dT0 = -2 r, dR/dT_k = 2 r, dR/db = 2 r m, dR/dG = -m m^T. */
static void residual_row(const ora_field *f, const double *T, int c, int code, ora_row *row)
{
    int i = c % f->nx, j = c / f->nx;
    double g[3], b[2];
    params_at(f, c, g, b);
    int dk[2];
    row->nd = donors_of(code, i, j, f->nx, row->d, dk);
    double T0 = T[c];
    if (row->nd == 2) {
        double m1x = -f->h * NBX[dk[0]], m1y = -f->h * NBY[dk[0]];
        double m2x = -f->h * NBX[dk[1]], m2y = -f->h * NBY[dk[1]];
        double E11 = gform(g, m1x, m1y, m1x, m1y);
        double E12 = gform(g, m1x, m1y, m2x, m2y);
        double E22 = gform(g, m2x, m2y, m2x, m2y);
        double det = E11 * E22 - E12 * E12;
        double Q11 = E22 / det, Q12 = -E12 / det, Q22 = E11 / det;
        double u1 = T[row->d[0]] + (m1x * b[0] + m1y * b[1]) - T0;
        double u2 = T[row->d[1]] + (m2x * b[0] + m2y * b[1]) - T0;
        double q1 = Q11 * u1 + Q12 * u2, q2 = Q12 * u1 + Q22 * u2; /* Q u */
        row->Jii = -2.0 * (q1 + q2);
        row->Jid[0] = 2.0 * q1;
        row->Jid[1] = 2.0 * q2;
        double px = m1x * q1 + m2x * q2, py = m1y * q1 + m2y * q2; /* Mst Q u */
        row->dRdb[0] = 2.0 * px;
        row->dRdb[1] = 2.0 * py;
        row->dRdG[0] = -px * px;
        row->dRdG[1] = -px * py;
        row->dRdG[2] = -py * py;
    } else if (row->nd == 1) {
        double mx = -f->h * NBX[dk[0]], my = -f->h * NBY[dk[0]];
        double r = T[row->d[0]] + (mx * b[0] + my * b[1]) - T0;
        row->Jii = -2.0 * r;
        row->Jid[0] = 2.0 * r;
        row->dRdb[0] = 2.0 * r * mx;
        row->dRdb[1] = 2.0 * r * my;
        row->dRdG[0] = -mx * mx;
        row->dRdG[1] = -mx * my;
        row->dRdG[2] = -my * my;
    }
}

/* ------------------------------------------------------------------------- */
/* Adjoint (Alg. backward; Eqs. implicit, param_grad, adjoint).                */
/* ------------------------------------------------------------------------- */

/* Vector-Jacobian product of the converged solve.
 *   g [n]       : dL/dT
 *   parent [n]  : active update codes (from ora_parents_levels)
 * Outputs dL/d(m11,m12,m22) as planes [3][n] with respect to the stored scalars
 * (the off-diagonal derivative counts both G12 and G21), dL/d(bx,by) as [2][n],
 * and dL/dt_s for each source. Nodes are visited by decreasing T; the adjoint
 * lambda_i = (g_i - sum_{j: i in donors(j)} J_ji lambda_j) / J_ii; then
 * dL/dtheta_i = -lambda_i dR_i/dtheta_i. Sources carry the residual
 * T_s - t_s, so J_ss = 1 and dL/dt_s = lambda_s. */
void ora_vjp(int nx, int ny, double h, const double *M, const double *om, int n_src,
             const int *src_idx, const double *T, const unsigned char *parent, const double *g,
             double *dM, double *dom, double *dsrc)
{
    ora_field f = {nx, ny, h, M, om};
    size_t n = (size_t)nx * ny;
    double *acc = (double *)calloc(n, sizeof(double)); /* sum_j J_ji lambda_j */
    double *lam = (double *)calloc(n, sizeof(double));
    memset(dM, 0, 3 * n * sizeof(double));
    memset(dom, 0, 2 * n * sizeof(double));
    size_t m;
    int *ord = sorted_reached(T, n, 1, &m);
    for (size_t q = 0; q < m; ++q) {
        int c = ord[q];
        int code = parent[c];
        if (code == ORA_SOURCE) {
            lam[c] = g[c] - acc[c];
            continue;
        }
        if (code >= 16) continue;
        ora_row row;
        residual_row(&f, T, c, code, &row);
        lam[c] = (g[c] - acc[c]) / row.Jii;
        for (int a = 0; a < row.nd; ++a) acc[row.d[a]] += row.Jid[a] * lam[c];
        dom[c] = -lam[c] * row.dRdb[0];
        dom[n + c] = -lam[c] * row.dRdb[1];
        dM[c] = -lam[c] * row.dRdG[0];
        dM[n + c] = -2.0 * lam[c] * row.dRdG[1];
        dM[2 * n + c] = -lam[c] * row.dRdG[2];
    }
    for (int s = 0; s < n_src; ++s) dsrc[s] = lam[src_idx[s]];
    free(ord);
    free(acc);
    free(lam);
}

/* Jacobian-vector product (forward mode; used to test the adjoint):
 * dT_i = -(dR_i/dtheta . dtheta_i + sum_k J_ik dT_k) / J_ii in increasing T,
 * dT_s = dt_s. dM/dom hold perturbations of the stored scalars. */
void ora_jvp(int nx, int ny, double h, const double *M, const double *om, int n_src,
             const int *src_idx, const double *T, const unsigned char *parent, const double *dMin,
             const double *domin, const double *dsrc, double *dT)
{
    ora_field f = {nx, ny, h, M, om};
    size_t n = (size_t)nx * ny;
    for (size_t c = 0; c < n; ++c) dT[c] = 0.0;
    for (int s = 0; s < n_src; ++s) dT[src_idx[s]] = dsrc ? dsrc[s] : 0.0;
    size_t m;
    int *ord = sorted_reached(T, n, 0, &m);
    for (size_t q = 0; q < m; ++q) {
        int c = ord[q];
        int code = parent[c];
        if (code >= 16) continue;
        ora_row row;
        residual_row(&f, T, c, code, &row);
        double rhs = row.dRdb[0] * domin[c] + row.dRdb[1] * domin[n + c] + row.dRdG[0] * dMin[c] +
                     2.0 * row.dRdG[1] * dMin[n + c] + row.dRdG[2] * dMin[2 * n + c];
        for (int a = 0; a < row.nd; ++a) rhs += row.Jid[a] * dT[row.d[a]];
        dT[c] = -rhs / row.Jii;
    }
    free(ord);
}

/* Value of one given candidate (code 0..7 two-point, 8..15 one-point) at node c
 * of the field T, for tests that accept any minimiser among near-equal
 * candidates. Returns +inf when a donor is missing or infinite; *valid tells
 * whether the candidate passes the validity and causality tests. */
double ora_candidate(int nx, int ny, double h, const double *M, const double *om, const double *T, int c,
                     int code, int *valid)
{
    ora_field f = {nx, ny, h, M, om};
    double g[3], b[2], Tn[8];
    params_at(&f, c, g, b);
    neighbour_times(&f, T, c % nx, c / nx, Tn);
    *valid = 0;
    if (code >= 8 && code < 16) {
        if (!isfinite(Tn[code - 8])) return INFINITY;
        *valid = 1;
        return one_point(g, b, h, code - 8, Tn[code - 8]);
    }
    if (code < 0 || code >= 8) return INFINITY;
    int kq = (code + 1) & 7;
    if (!isfinite(Tn[code]) || !isfinite(Tn[kq])) return INFINITY;
    double t;
    *valid = two_point(g, b, h, code, kq, Tn[code], Tn[kq], &t, NULL, NULL);
    return t;
}

/* ------------------------------------------------------------------------- */
/* Soft-min mode: the smooth alternative to stencil selection that the paper  */
/* names (Sec. 3.3, closing remarks on stencil boundaries).                   */
/* ------------------------------------------------------------------------- */
/* Each stencil k (neighbours k, k+1) contributes the minimum over its segment
 * of the Hopf-Lax objective: the two-point value when its barycentric
 * coordinates are both >= 0 (Eq. two_point; no causality test), else the
 * smaller one-point value of its finite endpoints (Eq. one_point). The node
 * takes the soft minimum T = -tau log sum_k exp(-H_k / tau) over the eight
 * stencils. Each H_k is continuously differentiable in its donor times and the
 * node's parameters (at the barycentric boundary the interior solution meets
 * the endpoint with the same derivatives), so T is too, and tau -> 0 gives the
 * minimum over all two-point and one-point values. */

/* H_k with its partial derivatives: dT[0], dT[1] with respect to the two donor
 * times, dth[5] with respect to the stored m11, m12, m22, bx, by. Returns
 * +inf (and zero partials) when neither donor is finite. */
static double stencil_hl(const double g[3], const double b[2], double h, int k, const double Tn[8], double dT[2],
                         double dth[5])
{
    int kq = (k + 1) & 7;
    dT[0] = dT[1] = 0.0;
    for (int a = 0; a < 5; ++a) dth[a] = 0.0;
    double best = INFINITY;
    int which = -1; /* 0: endpoint k, 1: endpoint kq, 2: interior */
    double lam[2] = {0.0, 0.0};
    if (isfinite(Tn[k]) && isfinite(Tn[kq])) {
        /* two_point leaves its outputs unwritten when the quadratic has no root */
        double t = INFINITY, l[2] = {-1.0, -1.0}, Qu[2];
        two_point(g, b, h, k, kq, Tn[k], Tn[kq], &t, l, Qu);
        if (isfinite(t) && l[0] >= 0.0 && l[1] >= 0.0) {
            best = t;
            which = 2;
            lam[0] = l[0];
            lam[1] = l[1];
        }
    }
    for (int e = 0; e < 2; ++e) {
        int kk = e == 0 ? k : kq;
        if (!isfinite(Tn[kk])) continue;
        double t = one_point(g, b, h, kk, Tn[kk]);
        if (t < best) {
            best = t;
            which = e;
        }
    }
    if (which < 0) return INFINITY;
    if (which < 2) {
        /* one-point from neighbour kk: T0 = T_kk + m.b + sqrt(m^T G m) */
        int kk = which == 0 ? k : kq;
        double mx = -h * NBX[kk], my = -h * NBY[kk];
        double e = sqrt(gform(g, mx, my, mx, my));
        dT[which] = 1.0;
        dth[0] = mx * mx / (2.0 * e);
        dth[1] = mx * my / e; /* the stored m12 enters G12 and G21 */
        dth[2] = my * my / (2.0 * e);
        dth[3] = mx;
        dth[4] = my;
        return best;
    }
    /* interior: residual R = u^T Q u - 1 with u = S - T0 1 and Q u = -lambda,
     * so dR/dT0 = 2 (l1 + l2), dR/dT_a = -2 l_a, dR/db = -2 Mst lambda,
     * dR/dG = -(Mst lambda)(Mst lambda)^T, and dT0/dx = -(dR/dx) / (dR/dT0) */
    double m1x = -h * NBX[k], m1y = -h * NBY[k], m2x = -h * NBX[kq], m2y = -h * NBY[kq];
    double dR0 = 2.0 * (lam[0] + lam[1]);
    double px = m1x * lam[0] + m2x * lam[1], py = m1y * lam[0] + m2y * lam[1];
    dT[0] = 2.0 * lam[0] / dR0;
    dT[1] = 2.0 * lam[1] / dR0;
    dth[0] = px * px / dR0;
    dth[1] = 2.0 * px * py / dR0;
    dth[2] = py * py / dR0;
    dth[3] = 2.0 * px / dR0;
    dth[4] = 2.0 * py / dR0;
    return best;
}

/* Soft update of node c: value, the derivatives coef[d] of that value with
 * respect to neighbour d's time (they sum to 1 over the finite neighbours),
 * and dth[5] with respect to the node's stored parameters. */
static double soft_local(const ora_field *f, const double *T, int c, double tau, double coef[8], double dth[5])
{
    double g[3], b[2], Tn[8], H[8], dTk[8][2], dthk[8][5];
    params_at(f, c, g, b);
    neighbour_times(f, T, c % f->nx, c / f->nx, Tn);
    double m = INFINITY;
    for (int k = 0; k < 8; ++k) {
        H[k] = stencil_hl(g, b, f->h, k, Tn, dTk[k], dthk[k]);
        if (H[k] < m) m = H[k];
    }
    for (int d = 0; d < 8; ++d) coef[d] = 0.0;
    for (int a = 0; a < 5; ++a) dth[a] = 0.0;
    if (!isfinite(m)) return INFINITY;
    double s = 0.0;
    for (int k = 0; k < 8; ++k)
        if (isfinite(H[k])) s += exp(-(H[k] - m) / tau);
    double v = m - tau * log(s);
    for (int k = 0; k < 8; ++k) {
        if (!isfinite(H[k])) continue;
        double p = exp(-(H[k] - v) / tau); /* softmax weight, sum 1 */
        coef[k] += p * dTk[k][0];
        coef[(k + 1) & 7] += p * dTk[k][1];
        for (int a = 0; a < 5; ++a) dth[a] += p * dthk[k][a];
    }
    return v;
}

/* Gauss-Seidel sweeps of the soft update in the four raster orderings, from
 * +inf (sources fixed at their times), until a full cycle changes no node by
 * more than tol relative. Returns 0 when converged, 1 at max_sweeps. */
int ora_soft_forward(int nx, int ny, double h, const double *M, const double *om, int n_src,
                     const int *src_idx, const double *src_t, double tau, int max_sweeps, double tol, double *T,
                     int *sweeps_out)
{
    ora_field f = {nx, ny, h, M, om};
    size_t n = (size_t)nx * ny;
    unsigned char *is_src = (unsigned char *)calloc(n, 1);
    for (size_t c = 0; c < n; ++c) T[c] = INFINITY;
    for (int s = 0; s < n_src; ++s) {
        is_src[src_idx[s]] = 1;
        T[src_idx[s]] = src_t ? src_t[s] : 0.0;
    }
    double coef[8], dth[5];
    int sweeps = 0, quiet = 0, status = 1;
    while (sweeps < max_sweeps) {
        int changed = 0, o = sweeps & 3;
        for (int jj = 0; jj < ny; ++jj) {
            int j = (o >= 2) ? ny - 1 - jj : jj;
            for (int ii = 0; ii < nx; ++ii) {
                int i = (o == 1 || o == 2) ? nx - 1 - ii : ii;
                int c = j * nx + i;
                if (is_src[c]) continue;
                double v = soft_local(&f, T, c, tau, coef, dth);
                if (counts_as_change(T[c], v, tol)) changed = 1;
                T[c] = v;
            }
        }
        ++sweeps;
        quiet = changed ? 0 : quiet + 1;
        if (quiet >= 4) {
            status = 0;
            break;
        }
    }
    if (sweeps_out) *sweeps_out = sweeps;
    free(is_src);
    return status;
}

/* The soft update's value and partial derivatives at node c of the field T. */
double ora_soft_local(int nx, int ny, double h, const double *M, const double *om, const double *T, double tau,
                      int c, double *coef, double *dth)
{
    ora_field f = {nx, ny, h, M, om};
    return soft_local(&f, T, c, tau, coef, dth);
}
