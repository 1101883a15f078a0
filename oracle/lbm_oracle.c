/*
 * Plain FP64 CPU oracle of the decoupled Hermite lattice Boltzmann scheme
 * (Hu, Zhang & Geng, "A decoupled scheme based on the Hermite expansion to
 * construct lattice Boltzmann models for the compressible Navier-Stokes
 * equations with arbitrary specific heat ratio", arXiv:1606.06107).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU library; it derives every lattice constant itself
 * from the quadrature conditions.
 *
 * Naming (the paper's letters -> this file):
 *   paper g_i (translational populations, streamed with xi_i)   -> f[i]
 *   paper h_j (rotational populations, advected with u)          -> g[j]
 *
 * Units: the paper's dimensionless units (Sec. II, theta = T, T0 = R_g = 1).
 * Lattice velocities xi_i = r * c_i with integer c_i; eta_j = r * j.
 * Grid spacing dx = 1 and time step dt = 1/r (so a population with velocity
 * xi_i moves c_i nodes per step; Sec. VI gives t = step / (X r)).  The BGK
 * factor is omega = 1/tau with tau counted in time steps, and the Courant
 * number of the rotational advection along axis a is nu_a = u_a / r.
 *
 * Everything is scalar loops over nodes and populations, FP64 throughout.
 * The node loop of a step may run under OpenMP: every node is computed from
 * the previous time level only, so the result does not depend on threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXQ 343

/* ---------------------------------------------------------------------- */
/* Lattices (Sec. IV, Tables I and II)                                     */
/* ---------------------------------------------------------------------- */

enum { ORC_D1Q7 = 1, ORC_D2Q49 = 2, ORC_D3Q343 = 3, ORC_D2Q37 = 4 };

/* (2k-1)!!: moment of order 2k of the unit Gaussian. */
static double gauss_moment(int order)
{
    if (order % 2) return 0.0;
    double m = 1.0;
    for (int k = order - 1; k > 0; k -= 2) m *= k;
    return m;
}

/* Solve the dense system A x = b (n <= 8) by Gaussian elimination with
 * partial pivoting.  A is row-major and is overwritten. */
static int solve_dense(int n, double *A, double *b, double *x)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
        if (A[piv * n + col] == 0.0) return -1;
        if (piv != col) {
            for (int k = 0; k < n; ++k) {
                double t = A[col * n + k];
                A[col * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double f = A[r * n + col] / A[col * n + col];
            for (int k = col; k < n; ++k) A[r * n + k] -= f * A[col * n + k];
            b[r] -= f * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
        x[r] = s / A[r * n + r];
    }
    return 0;
}

/* D1Q7 weights at scaling factor r from the even moment conditions of order
 * 2, 4, 6 (the unknowns are w_1, w_2, w_3; w_0 closes the zeroth moment). */
static void d1q7_weights(double r, double w[4])
{
    double A[9], b[3], x[3];
    for (int m = 0; m < 3; ++m) {
        int p = 2 * (m + 1);
        for (int k = 1; k <= 3; ++k) A[m * 3 + (k - 1)] = 2.0 * pow(r * k, p);
        b[m] = gauss_moment(p);
    }
    solve_dense(3, A, b, x);
    w[1] = x[0]; w[2] = x[1]; w[3] = x[2];
    w[0] = 1.0 - 2.0 * (x[0] + x[1] + x[2]);
}

/* Residual of the eighth moment; its root near 1.197 is the scaling factor
 * of the univariate 7-point Gauss-Hermite model (Table II). */
static double d1q7_m8_residual(double r)
{
    double w[4];
    d1q7_weights(r, w);
    double m = 0.0;
    for (int k = 1; k <= 3; ++k) m += 2.0 * w[k] * pow(r * k, 8);
    return m - 105.0;
}

/* Scaling factor r by bisection on [1.15, 1.25] (the residual changes sign
 * once there), refined to the last bit. */
double orc_d1q7_r(void)
{
    double lo = 1.15, hi = 1.25;
    double flo = d1q7_m8_residual(lo);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        double fm = d1q7_m8_residual(mid);
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* D2Q37 of Table I with the multiplicities read as 1,4,4,4,8,4,8,4 (groups
 * Perm(2r,r) and Perm(3r,r) hold eight velocities).  Weights solve the even
 * moment conditions of total order 0..8 of a 2-D unit Gaussian at the D1Q7
 * scaling factor (Sec. IV requires a common r).  The nine conditions have
 * rank eight at this r; eight of them (all but x^4) fix the weights and the
 * tests check the ninth. */
static const int d2q37_group[8][2] = {
    {0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {3, 0}, {3, 1}, {3, 3}};

static void d2q37_weights(double r, double wg[8])
{
    /* conditions (a,b): sum_i w_i cx^(2a) cy^(2b) r^(2a+2b) = (2a-1)!!(2b-1)!! */
    static const int cond[8][2] = {{0, 0}, {1, 0}, {1, 1}, {3, 0},
                                   {2, 1}, {4, 0}, {3, 1}, {2, 2}};
    double A[64], b[8];
    for (int m = 0; m < 8; ++m) {
        int a = cond[m][0], bb = cond[m][1];
        for (int gI = 0; gI < 8; ++gI) {
            /* sum over the members of the group (all sign/axis permutations) */
            int p = d2q37_group[gI][0], q = d2q37_group[gI][1];
            int mem[8][2], nm = 0;
            int base[2][2] = {{p, q}, {q, p}};
            for (int s = 0; s < 2; ++s)
                for (int sx = -1; sx <= 1; sx += 2)
                    for (int sy = -1; sy <= 1; sy += 2) {
                        int cx = sx * base[s][0], cy = sy * base[s][1];
                        int dup = 0;
                        for (int k = 0; k < nm; ++k)
                            if (mem[k][0] == cx && mem[k][1] == cy) dup = 1;
                        if (!dup) { mem[nm][0] = cx; mem[nm][1] = cy; ++nm; }
                    }
            double s = 0.0;
            for (int k = 0; k < nm; ++k)
                s += pow(r * mem[k][0], 2 * a) * pow(r * mem[k][1], 2 * bb);
            A[m * 8 + gI] = s;
        }
        b[m] = gauss_moment(2 * a) * gauss_moment(2 * bb);
    }
    solve_dense(8, A, b, wg);
}

/* Fill velocities c[Q][3] (integers stored as int) and weights w[Q].
 * Returns Q, or -1 for an unknown kind.  Index order for the tensor lattices:
 * i = cx+3 (1-D), (cy+3)*7 + cx+3 (2-D), ((cz+3)*7 + cy+3)*7 + cx+3 (3-D). */
int orc_lattice(int kind, int *c, double *w, double *r_out)
{
    double r = orc_d1q7_r();
    double w1[4];
    d1q7_weights(r, w1);
    if (r_out) *r_out = r;
    int Q = 0;
    if (kind == ORC_D1Q7 || kind == ORC_D2Q49 || kind == ORC_D3Q343) {
        int D = (kind == ORC_D1Q7) ? 1 : (kind == ORC_D2Q49) ? 2 : 3;
        int nz = D >= 3 ? 7 : 1, ny = D >= 2 ? 7 : 1;
        for (int kz = 0; kz < nz; ++kz)
            for (int ky = 0; ky < ny; ++ky)
                for (int kx = 0; kx < 7; ++kx) {
                    int cx = kx - 3, cy = D >= 2 ? ky - 3 : 0, cz = D >= 3 ? kz - 3 : 0;
                    c[Q * 3 + 0] = cx; c[Q * 3 + 1] = cy; c[Q * 3 + 2] = cz;
                    double ww = w1[abs(cx)];
                    if (D >= 2) ww *= w1[abs(cy)];
                    if (D >= 3) ww *= w1[abs(cz)];
                    w[Q] = ww;
                    ++Q;
                }
        return Q;
    }
    if (kind == ORC_D2Q37) {
        double wg[8];
        d2q37_weights(r, wg);
        for (int gI = 0; gI < 8; ++gI) {
            int p = d2q37_group[gI][0], q = d2q37_group[gI][1];
            int base[2][2] = {{p, q}, {q, p}};
            int start = Q;
            for (int s = 0; s < 2; ++s)
                for (int sx = -1; sx <= 1; sx += 2)
                    for (int sy = -1; sy <= 1; sy += 2) {
                        int cx = sx * base[s][0], cy = sy * base[s][1];
                        int dup = 0;
                        for (int k = start; k < Q; ++k)
                            if (c[k * 3] == cx && c[k * 3 + 1] == cy) dup = 1;
                        if (!dup) {
                            c[Q * 3 + 0] = cx; c[Q * 3 + 1] = cy; c[Q * 3 + 2] = 0;
                            w[Q] = wg[gI];
                            ++Q;
                        }
                    }
        }
        return Q;
    }
    return -1;
}

/* Rotational lattice D1Q7: eta_j = r*(j-3), same r as the translational
 * lattice (Sec. IV: the two models must share the scaling factor). */
static void rot_lattice(double *eta, double *w)
{
    double r = orc_d1q7_r();
    double w1[4];
    d1q7_weights(r, w1);
    for (int j = 0; j < 7; ++j) {
        eta[j] = r * (j - 3);
        w[j] = w1[abs(j - 3)];
    }
}

/* ---------------------------------------------------------------------- */
/* Equilibria (Sec. IV)                                                    */
/* ---------------------------------------------------------------------- */

/* Translational equilibrium: fourth-order Hermite expansion of the
 * Maxwellian g^eq(xi) of Sec. II, w_i rho sum_k a^(k).H^(k)(xi_i) / k!, with
 * the Hermite coefficients of a Maxwellian of velocity u and temperature
 * theta contracted with the Hermite tensors (xi.u = a, |xi|^2 = xi2, D the
 * spatial dimension of the lattice). */
void orc_feq(int D, int Q, const int *c, const double *w, double r,
             double rho, const double *u, double theta, double *out)
{
    double u2 = 0.0;
    for (int d = 0; d < D; ++d) u2 += u[d] * u[d];
    double th1 = theta - 1.0;
    for (int i = 0; i < Q; ++i) {
        double a = 0.0, xi2 = 0.0;
        for (int d = 0; d < D; ++d) {
            double xi = r * c[i * 3 + d];
            a += xi * u[d];
            xi2 += xi * xi;
        }
        double H0 = 1.0;
        double H1 = a;
        double H2 = a * a - u2 + th1 * (xi2 - D);
        double H3 = a * (a * a - 3.0 * u2 + 3.0 * th1 * (xi2 - D - 2.0));
        double H4 = a * a * a * a - 6.0 * a * a * u2 + 3.0 * u2 * u2
                  + 6.0 * th1 * (a * a * (xi2 - D - 4.0) + (D + 2.0 - xi2) * u2)
                  + 3.0 * th1 * th1 * (xi2 * xi2 - 2.0 * (D + 2.0) * xi2 + D * (D + 2.0));
        out[i] = w[i] * rho * (H0 + H1 + H2 / 2.0 + H3 / 6.0 + H4 / 24.0);
    }
}

/* Rotational equilibrium: fourth-order Hermite expansion of the normalised
 * 1-D Gaussian h^eq(eta) of variance theta (zero mean, so the odd terms
 * vanish; the expansion is one-dimensional). */
static void geq_on(const double *eta, const double *w, double theta, double *out)
{
    double th1 = theta - 1.0;
    for (int j = 0; j < 7; ++j) {
        double e2 = eta[j] * eta[j];
        double H2 = th1 * (e2 - 1.0);
        double H4 = 3.0 * th1 * th1 * (e2 * e2 - 6.0 * e2 + 3.0);
        out[j] = w[j] * (1.0 + H2 / 2.0 + H4 / 24.0);
    }
}

void orc_geq(double theta, double *out)
{
    double eta[7], w[7];
    rot_lattice(eta, w);
    geq_on(eta, w, theta, out);
}

/* ---------------------------------------------------------------------- */
/* Grid, moments and the time step (Sec. V)                                */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t dim;        /* spatial dimension D = 1, 2, 3 */
    int32_t lattice;    /* ORC_D1Q7, ORC_D2Q49, ORC_D3Q343, ORC_D2Q37 */
    int64_t n[3];       /* nodes per axis, unused axes = 1 */
    int32_t bc[3];      /* 0 = periodic, 1 = open (zero-gradient clamp) */
    double n_rot;       /* rotational degrees of freedom n */
    double tau;         /* relaxation time in time steps of the streaming update */
    double fd_courant;  /* 0: collide-and-stream update of the translational
                           populations (reading A); lambda > 0: the finite-difference
                           update written in Sec. V A (reading B) with time step
                           lambda / r, i.e. lambda times the streaming step */
    int32_t g_substeps; /* <= 1: the rotational update of Sec. V A as written;
                           m > 1: its advection in m sub-steps of Courant number
                           nu_a / m (relaxation once per step), a device outside
                           the paper used to tell the advection's Courant limit
                           from other causes of divergence */
} orc_grid;

typedef struct {
    int D, Q;
    int c[ORC_MAXQ * 3];
    double w[ORC_MAXQ];
    double r;
    double eta[7], wr[7];
} lat_t;

static int make_lat(const orc_grid *G, lat_t *L)
{
    L->D = G->dim;
    L->Q = orc_lattice(G->lattice, L->c, L->w, &L->r);
    rot_lattice(L->eta, L->wr);
    int want = (G->lattice == ORC_D1Q7) ? 1 : (G->lattice == ORC_D3Q343) ? 3 : 2;
    return (L->Q > 0 && want == G->dim) ? 0 : -1;
}

static int64_t nnodes(const orc_grid *G) { return G->n[0] * G->n[1] * G->n[2]; }

/* Neighbour index along one axis: periodic wrap or clamp to [0, n-1]. */
static int64_t wrap_or_clamp(int64_t x, int64_t n, int bc)
{
    if (bc == 0) {
        x %= n;
        if (x < 0) x += n;
        return x;
    }
    if (x < 0) return 0;
    if (x >= n) return n - 1;
    return x;
}

/* Moments of one node, Sec. V B steps (3) and (4):
 *   rho = sum f_i, rho u = sum f_i xi_i, E_t = sum f_i |xi_i|^2 / 2,
 *   e_r = sum_j (n/2) g_j eta_j^2,
 *   T = 2/(D+n) (E_t + rho e_r - rho |u|^2 / 2) / rho. */
static void node_moments(const lat_t *L, double n_rot, const double *fn, const double *gn,
                         double *rho, double *u, double *T, double *Etot)
{
    double m0 = 0.0, m1[3] = {0, 0, 0}, et = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        double xi2 = 0.0;
        for (int d = 0; d < L->D; ++d) {
            double xi = L->r * L->c[i * 3 + d];
            m1[d] += fn[i] * xi;
            xi2 += xi * xi;
        }
        m0 += fn[i];
        et += fn[i] * 0.5 * xi2;
    }
    double er = 0.0;
    for (int j = 0; j < 7; ++j) er += 0.5 * n_rot * gn[j] * L->eta[j] * L->eta[j];
    double u2 = 0.0;
    for (int d = 0; d < L->D; ++d) {
        u[d] = m1[d] / m0;
        u2 += u[d] * u[d];
    }
    *rho = m0;
    *T = 2.0 / (L->D + n_rot) * (et + m0 * er - 0.5 * m0 * u2) / m0;
    if (Etot) *Etot = et + m0 * er;
}

/* Populations at equilibrium with the given fields (the initial condition). */
int orc_init_eq(const orc_grid *G, const double *rho, const double *u, const double *T,
                double *f, double *g)
{
    lat_t L;
    if (make_lat(G, &L)) return -1;
    int64_t N = nnodes(G);
    double fe[ORC_MAXQ], ge[7], un[3];
    for (int64_t x = 0; x < N; ++x) {
        for (int d = 0; d < L.D; ++d) un[d] = u[d * N + x];
        orc_feq(L.D, L.Q, L.c, L.w, L.r, rho[x], un, T[x], fe);
        geq_on(L.eta, L.wr, T[x], ge);
        for (int i = 0; i < L.Q; ++i) f[i * N + x] = fe[i];
        for (int j = 0; j < 7; ++j) g[j * N + x] = ge[j];
    }
    return 0;
}

/* Third-order upwind difference of Sec. V A along one axis at node p, for
 * Courant number of sign s.  For s >= 0:
 *   (h[x-2] - 6 h[x-1] + 3 h[x] + 2 h[x+1]) / 6,
 * for s < 0:
 *   (-h[x+2] + 6 h[x+1] - 3 h[x] - 2 h[x-1]) / 6,
 * with neighbours wrapped (periodic) or clamped (open). */
static double upwind3(const orc_grid *G, const double *h, const int64_t xyz[3], int axis,
                      double s)
{
    int64_t N0 = G->n[0], N1 = G->n[1];
    double v[5];
    for (int k = -2; k <= 2; ++k) {
        int64_t q[3] = {xyz[0], xyz[1], xyz[2]};
        q[axis] = wrap_or_clamp(q[axis] + k, G->n[axis], G->bc[axis]);
        v[k + 2] = h[q[0] + N0 * (q[1] + N1 * q[2])];
    }
    if (s >= 0.0)
        return (v[0] - 6.0 * v[1] + 3.0 * v[2] + 2.0 * v[3]) / 6.0;
    return (-v[4] + 6.0 * v[3] - 3.0 * v[2] - 2.0 * v[1]) / 6.0;
}

/* One time step of Sec. V (collide-and-stream reading of the update of the
 * translational populations; forward-Euler upwind update of the rotational
 * populations with the fluid velocity).  Both updates use the moments of the
 * state at time t.  f, g hold time t on entry and t+1 on exit; fs, gs are
 * scratch of the same sizes. */
static void one_step(const orc_grid *G, const lat_t *L, double *f, double *g, double *fs,
                     double *gs)
{
    int64_t N = nnodes(G);
    double omega = 1.0 / G->tau;
    int64_t N0 = G->n[0], N1 = G->n[1];

#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double fn[ORC_MAXQ], gn[7], fe[ORC_MAXQ], ge[7], u[3], rho, T;
        for (int i = 0; i < L->Q; ++i) fn[i] = f[i * N + x];
        for (int j = 0; j < 7; ++j) gn[j] = g[j * N + x];
        node_moments(L, G->n_rot, fn, gn, &rho, u, &T, NULL);
        orc_feq(L->D, L->Q, L->c, L->w, L->r, rho, u, T, fe);
        geq_on(L->eta, L->wr, T, ge);
        /* BGK relaxation of the translational populations (post-collision). */
        for (int i = 0; i < L->Q; ++i) fs[i * N + x] = fn[i] - omega * (fn[i] - fe[i]);
        /* Rotational populations: advect with u (Courant nu_a = u_a / r), relax. */
        int64_t xyz[3] = {x % N0, (x / N0) % N1, x / (N0 * N1)};
        for (int j = 0; j < 7; ++j) {
            double adv = 0.0;
            for (int a = 0; a < L->D; ++a) {
                double nu = u[a] / L->r;
                adv += nu * upwind3(G, g + j * N, xyz, a, nu);
            }
            gs[j * N + x] = gn[j] - adv - omega * (gn[j] - ge[j]);
        }
    }
    /* Streaming, written as a pull: f_i(x, t+1) = f*_i(S(x - c_i)) with S the
     * periodic wrap or the open-boundary clamp of each axis. */
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        int64_t xyz[3] = {x % N0, (x / N0) % N1, x / (N0 * N1)};
        for (int i = 0; i < L->Q; ++i) {
            int64_t q[3];
            for (int d = 0; d < 3; ++d) {
                int cd = (d < L->D) ? L->c[i * 3 + d] : 0;
                q[d] = wrap_or_clamp(xyz[d] - cd, G->n[d], G->bc[d]);
            }
            f[i * N + x] = fs[i * N + q[0] + N0 * (q[1] + N1 * q[2])];
        }
        for (int j = 0; j < 7; ++j) g[j * N + x] = gs[j * N + x];
    }
}

/* One time step of the finite-difference form of Sec. V A for both kinds of
 * population (reading B of the translational update): with time step
 * dt = lambda / r (lambda = G->fd_courant) and dx = 1,
 *   f_i(x, t+dt) = f_i - sum_a (lambda c_ia) D_a[f_i] - (lambda/tau) (f_i - f_i^eq)
 *   g_j(x, t+dt) = g_j - sum_a (lambda u_a / r) D_a[g_j] - (lambda/tau) (g_j - g_j^eq)
 * where D_a is the third-order upwind difference along axis a oriented by the
 * sign of the Courant number (xi_ia dt / dx = lambda c_ia for f, u_a dt / dx
 * for g), every term evaluated at time t (forward Euler), and tau the
 * relaxation time in streaming steps (1/r), so the collision term is dt/tau
 * in time units.  lambda = 1 is the time step of the streaming update. */
static void one_step_fd(const orc_grid *G, const lat_t *L, double *f, double *g, double *fs,
                        double *gs)
{
    int64_t N = nnodes(G);
    const double lam = G->fd_courant;
    const double omega = lam / G->tau;
    int64_t N0 = G->n[0], N1 = G->n[1];

#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double fn[ORC_MAXQ], gn[7], fe[ORC_MAXQ], ge[7], u[3], rho, T;
        for (int i = 0; i < L->Q; ++i) fn[i] = f[i * N + x];
        for (int j = 0; j < 7; ++j) gn[j] = g[j * N + x];
        node_moments(L, G->n_rot, fn, gn, &rho, u, &T, NULL);
        orc_feq(L->D, L->Q, L->c, L->w, L->r, rho, u, T, fe);
        geq_on(L->eta, L->wr, T, ge);
        int64_t xyz[3] = {x % N0, (x / N0) % N1, x / (N0 * N1)};
        for (int i = 0; i < L->Q; ++i) {
            double adv = 0.0;
            for (int a = 0; a < L->D; ++a) {
                double nu = lam * L->c[i * 3 + a];
                if (nu != 0.0) adv += nu * upwind3(G, f + i * N, xyz, a, nu);
            }
            fs[i * N + x] = fn[i] - adv - omega * (fn[i] - fe[i]);
        }
        for (int j = 0; j < 7; ++j) {
            double adv = 0.0;
            for (int a = 0; a < L->D; ++a) {
                double nu = lam * u[a] / L->r;
                adv += nu * upwind3(G, g + j * N, xyz, a, nu);
            }
            gs[j * N + x] = gn[j] - adv - omega * (gn[j] - ge[j]);
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        for (int i = 0; i < L->Q; ++i) f[i * N + x] = fs[i * N + x];
        for (int j = 0; j < 7; ++j) g[j * N + x] = gs[j * N + x];
    }
}

/* One time step with the rotational advection split into m sub-steps:
 * g(t+1) = A^m g(t) - omega (g(t) - g^eq(T)), where A is the forward-Euler
 * upwind advection of Sec. V A with Courant numbers nu_a / m and the fluid
 * velocity of time t.  For m = 1 this is the update of one_step.  u: N*3
 * scratch, gt: 7*N scratch. */
static void one_step_sub(const orc_grid *G, const lat_t *L, double *f, double *g, double *fs,
                         double *gs, int m, double *u3, double *gt)
{
    int64_t N = nnodes(G);
    double omega = 1.0 / G->tau;
    int64_t N0 = G->n[0], N1 = G->n[1];
    for (int64_t x = 0; x < N; ++x) {
        double fn[ORC_MAXQ], gn[7], fe[ORC_MAXQ], ge[7], u[3] = {0, 0, 0}, rho, T;
        for (int i = 0; i < L->Q; ++i) fn[i] = f[i * N + x];
        for (int j = 0; j < 7; ++j) gn[j] = g[j * N + x];
        node_moments(L, G->n_rot, fn, gn, &rho, u, &T, NULL);
        orc_feq(L->D, L->Q, L->c, L->w, L->r, rho, u, T, fe);
        geq_on(L->eta, L->wr, T, ge);
        for (int i = 0; i < L->Q; ++i) fs[i * N + x] = fn[i] - omega * (fn[i] - fe[i]);
        for (int j = 0; j < 7; ++j) gs[j * N + x] = omega * (gn[j] - ge[j]);  /* relaxation term */
        for (int d = 0; d < 3; ++d) u3[d * N + x] = u[d];
    }
    for (int s = 0; s < m; ++s) {
        for (int64_t x = 0; x < N; ++x) {
            int64_t xyz[3] = {x % N0, (x / N0) % N1, x / (N0 * N1)};
            for (int j = 0; j < 7; ++j) {
                double adv = 0.0;
                for (int a = 0; a < L->D; ++a) {
                    double nu = u3[a * N + x] / L->r / m;
                    adv += nu * upwind3(G, g + j * N, xyz, a, nu);
                }
                gt[j * N + x] = g[j * N + x] - adv;
            }
        }
        memcpy(g, gt, sizeof(double) * 7 * (size_t)N);
    }
    for (int64_t x = 0; x < N; ++x) {
        int64_t xyz[3] = {x % N0, (x / N0) % N1, x / (N0 * N1)};
        for (int i = 0; i < L->Q; ++i) {
            int64_t q[3];
            for (int d = 0; d < 3; ++d) {
                int cd = (d < L->D) ? L->c[i * 3 + d] : 0;
                q[d] = wrap_or_clamp(xyz[d] - cd, G->n[d], G->bc[d]);
            }
            f[i * N + x] = fs[i * N + q[0] + N0 * (q[1] + N1 * q[2])];
        }
        for (int j = 0; j < 7; ++j) g[j * N + x] -= gs[j * N + x];
    }
}

/* Advance nsteps time steps in place.  fs/gs: caller scratch, same sizes as f/g. */
int orc_step(const orc_grid *G, double *f, double *g, double *fs, double *gs, int64_t nsteps)
{
    lat_t L;
    if (make_lat(G, &L)) return -1;
    if (G->fd_courant < 0.0) return -3;
    if (G->fd_courant > 0.0) {
        if (G->tau <= 0.0) return -2;
        for (int64_t s = 0; s < nsteps; ++s) one_step_fd(G, &L, f, g, fs, gs);
        return 0;
    }
    if (G->tau <= 0.5) return -2;
    if (G->g_substeps > 1) {
        int64_t N = nnodes(G);
        double *u3 = (double *)malloc(sizeof(double) * 3 * (size_t)N);
        double *gt = (double *)malloc(sizeof(double) * 7 * (size_t)N);
        if (!u3 || !gt) {
            free(u3);
            free(gt);
            return -4;
        }
        for (int64_t s = 0; s < nsteps; ++s) one_step_sub(G, &L, f, g, fs, gs, G->g_substeps, u3, gt);
        free(u3);
        free(gt);
        return 0;
    }
    for (int64_t s = 0; s < nsteps; ++s) one_step(G, &L, f, g, fs, gs);
    return 0;
}

/* Macroscopic fields and totals of the state (f, g): rho[N], u[D][N], T[N]
 * (any may be NULL), totals[2+D] = {mass, momentum[D], energy} with energy
 * = sum over nodes of E_t + rho e_r, summed in node order. */
int orc_moments(const orc_grid *G, const double *f, const double *g, double *rho,
                double *u, double *T, double *totals)
{
    lat_t L;
    if (make_lat(G, &L)) return -1;
    int64_t N = nnodes(G);
    double M = 0.0, P[3] = {0, 0, 0}, E = 0.0;
    double fn[ORC_MAXQ], gn[7];
    for (int64_t x = 0; x < N; ++x) {
        double r_, u_[3], T_, Et;
        for (int i = 0; i < L.Q; ++i) fn[i] = f[i * N + x];
        for (int j = 0; j < 7; ++j) gn[j] = g[j * N + x];
        node_moments(&L, G->n_rot, fn, gn, &r_, u_, &T_, &Et);
        if (rho) rho[x] = r_;
        if (T) T[x] = T_;
        for (int d = 0; d < L.D; ++d) {
            if (u) u[d * N + x] = u_[d];
            P[d] += r_ * u_[d];
        }
        M += r_;
        E += Et;
    }
    if (totals) {
        totals[0] = M;
        for (int d = 0; d < L.D; ++d) totals[1 + d] = P[d];
        totals[1 + L.D] = E;
    }
    return 0;
}

/* Thread count of the node loops (1 = serial).  Returns the count in use. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
