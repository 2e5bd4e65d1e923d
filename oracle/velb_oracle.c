/*
 * Plain FP64 CPU oracle for the viscoelastic immersed-boundary lattice Boltzmann step of
 * Floyd, Vaikuntanathan and Dinner, arXiv 2209.14889.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously-correct reference the GPU library is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg load it.  It
 * shares no code with the GPU library.
 *
 * Every step takes the fields at time t as inputs (Fig. 2 caption: all fields are updated from
 * the previous time step, so the order of the updates does not matter).  One step is done as
 * separate whole-field passes, in this order:
 *   1. node forces of every immersed body (App. A, eqConst and the spring/bending potentials),
 *      plus the constant pull shared equally by the nodes;
 *   2. spreading of the node forces with the cosine kernel (App. A);
 *   3. divergence of the polymer stress, f^p = div sigma^p (Sec. II B);
 *   4. molecular field h(P), Ericksen stress sigma^E and f^E = div sigma^E (Sec. II C 1);
 *   5. moments rho = sum h, rho v = sum c h + F/2 (eqrhoDef, eqvDef with Guo's half-force);
 *   6. BGK collision (eqBGK) with the standard second-order D2Q9 equilibrium and Guo forcing;
 *   7. streaming (eqLB), periodic, or halfway bounce-back at walls (App. C boundary text);
 *   8. velocity gradient, its symmetric part Psi and vorticity Omega (Sec. II B);
 *   9. stiffness C~(P) from the von Mises closure (eqPk) and the App. B closed form;
 *  10. Heun (predictor-corrector) step of the tensorial stress equation eqStiffCons with the
 *      corotational derivative;
 *  11. Heun step of the Beris-Edwards equation eqBE with the molecular field of eqFfunctional;
 *  12. Heun step of the overdamped no-slip node motion dR/dt = v(R) (App. A).
 *
 * Readings where the paper is silent (all listed in the design notes of the repository):
 *   - second-order central differences for gradients and divergences, 5-point Laplacian,
 *     central advection;
 *   - Heun keeps every cross-field input (v, grad v, C~, F) frozen at time t and re-evaluates
 *     only the field's own value at the predicted state;
 *   - the Ericksen gradient term carries the coefficient kappa of the free energy;
 *   - the App. B matrix acts on plain tensor components (Xxx, Xyy, Xxy);
 *   - the k-bracket of App. B equals k^3 I4(k) and is evaluated as such;
 *   - fluid velocity for finite differences and the immersed boundary is (sum c h + F/2)/rho.
 */
#include "velb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 lattice: rest, 4 axis links, 4 diagonal links */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------------------------------ */
/* field access with the boundary rules                                                        */
/* ------------------------------------------------------------------------------------------ */

static inline int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

enum { GHOST_EVEN = 0, GHOST_ODD = 1 };

/* value of plane f at (x, y).  Periodic directions wrap.  Beyond a wall (y with walls >= 1, x
 * with walls == 2) the ghost mirrors the first interior row or column: EVEN for
 * zero-normal-derivative fields (stress, polarization, App. C), ODD for the velocity (no-slip wall
 * half way between the sites). */
static inline double at(const orc_params *p, const double *f, int x, int y, int ghost) {
    double sign = 1.0;
    if (p->walls == 2 && (x < 0 || x >= p->nx)) {
        x = x < 0 ? -1 - x : 2 * p->nx - 1 - x;
        if (ghost == GHOST_ODD) sign = -sign;
    } else {
        x = wrap(x, p->nx);
    }
    if (p->walls && (y < 0 || y >= p->ny)) {
        y = y < 0 ? -1 - y : 2 * p->ny - 1 - y;
        if (ghost == GHOST_ODD) sign = -sign;
    } else {
        y = wrap(y, p->ny);
    }
    return sign * f[(size_t)y * p->nx + x];
}

static inline double ddx(const orc_params *p, const double *f, int x, int y, int g) {
    return 0.5 * (at(p, f, x + 1, y, g) - at(p, f, x - 1, y, g));
}
static inline double ddy(const orc_params *p, const double *f, int x, int y, int g) {
    return 0.5 * (at(p, f, x, y + 1, g) - at(p, f, x, y - 1, g));
}
static inline double lap5(const orc_params *p, const double *f, int x, int y, int g) {
    return at(p, f, x + 1, y, g) + at(p, f, x - 1, y, g) + at(p, f, x, y + 1, g) +
           at(p, f, x, y - 1, g) - 4.0 * at(p, f, x, y, g);
}

/* ------------------------------------------------------------------------------------------ */
/* von Mises closure and the stiffness tensor (Sec. II C 3, eqPk, App. B)                      */
/* ------------------------------------------------------------------------------------------ */

/* I_n(k) = sum_m (k/2)^(2m+n) / (m! (m+n)!), every term positive */
double orc_bessel_i(int n, double k) {
    if (k == 0.0) return n == 0 ? 1.0 : 0.0;
    double hk = 0.5 * k, q = hk * hk;
    double t = 1.0;
    for (int i = 1; i <= n; ++i) t *= hk / i;
    double sum = t;
    for (int m = 1; m < 2000; ++m) {
        t *= q / ((double)m * (double)(m + n));
        sum += t;
        if (t < 1e-18 * sum && m > hk) break;
    }
    return sum;
}

static double mean_cos(double k) { return k == 0.0 ? 0.0 : orc_bessel_i(1, k) / orc_bessel_i(0, k); }

/* solve I1(k)/I0(k) = p by Newton's method kept inside a shrinking bracket.  The starting value
 * is the approximate inverse of Best and Fisher (1981). */
double orc_k_of_p(double p) {
    if (p <= 0.0) return 0.0;
    if (p >= 1.0) return INFINITY;
    double k;
    if (p < 0.53)
        k = 2.0 * p + p * p * p + 5.0 * pow(p, 5) / 6.0;
    else if (p < 0.85)
        k = -0.4 + 1.39 * p + 0.43 / (1.0 - p);
    else
        k = 1.0 / (p * p * p - 4.0 * p * p + 3.0 * p);
    double lo = 0.0, hi = 2.0 * k + 1.0;
    while (mean_cos(hi) < p) hi *= 2.0;
    if (k <= lo || k >= hi) k = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double A = mean_cos(k);
        double f = A - p;
        if (f > 0.0) hi = k; else lo = k;
        double dA = 1.0 - A / k - A * A;          /* d/dk of I1/I0 */
        double kn = k - f / dA;
        if (!(kn > lo && kn < hi)) kn = 0.5 * (lo + hi);
        if (fabs(kn - k) <= 1e-15 * (k > 1.0 ? k : 1.0)) { k = kn; break; }
        k = kn;
    }
    return k;
}

void orc_stiffness(double Px, double Py, const double Kx[4], double P_clamp, double C[9]) {
    const double K1111 = Kx[0], K1122 = Kx[1], K2222 = Kx[2], K1212 = Kx[3];
    double P = sqrt(Px * Px + Py * Py);
    double Pk = P < P_clamp ? P : P_clamp;          /* clamp only the magnitude fed to k */
    double k = orc_k_of_p(Pk);
    double I0 = orc_bessel_i(0, k);
    double I2 = orc_bessel_i(2, k);
    double I4 = orc_bessel_i(4, k);                  /* = (k(k^2+24) I0 - 8(k^2+6) I1) / k^3 */
    double thP = atan2(Py, Px);                      /* polar angle of P-hat */
    double c2 = cos(2.0 * thP), s2 = sin(2.0 * thP);
    double c4 = cos(4.0 * thP), s4 = sin(4.0 * thP);
    double A = K1111 - 2.0 * K1122 - 4.0 * K1212 + K2222;
    double B = K1111 - K2222;
    double C11 = (I4 * c4 * A + I0 * (3.0 * K1111 + 2.0 * K1122 + 4.0 * K1212 + 3.0 * K2222) +
                  4.0 * I2 * B * c2) / (8.0 * I0);
    double C12 = (-I4 * c4 * A / I0 + K1111 + 6.0 * K1122 - 4.0 * K1212 + K2222) / 8.0;
    double C13 = (M_PI * I4 * s4 * A + 2.0 * M_PI * I2 * B * s2) / (4.0 * M_PI * I0);
    double C22 = C11 - I2 * B * c2 / I0;
    double C23 = -(M_PI * I4 * s4 * A + 2.0 * M_PI * I2 * (K2222 - K1111) * s2) / (4.0 * M_PI * I0);
    double C31 = (M_PI * I4 * s4 * A + 2.0 * M_PI * I2 * B * s2) / (8.0 * M_PI * I0);
    double C32 = -(M_PI * I4 * s4 * A + 2.0 * M_PI * I2 * (K2222 - K1111) * s2) / (8.0 * M_PI * I0);
    double C33 = (-I4 * c4 * A / I0 + K1111 - 2.0 * K1122 + 4.0 * K1212 + K2222) / 4.0;
    C[0] = C11; C[1] = C12; C[2] = C13;
    C[3] = C12; C[4] = C22; C[5] = C23;
    C[6] = C31; C[7] = C32; C[8] = C33;
}

/* ------------------------------------------------------------------------------------------ */
/* immersed boundary (App. A)                                                                  */
/* ------------------------------------------------------------------------------------------ */

double orc_phi(double r) {
    double a = fabs(r);
    return a < 2.0 ? 0.25 * (1.0 + cos(M_PI * r / 2.0)) : 0.0;
}

double orc_body_energy(const orc_body *b) {
    int n = b->n;
    const double *R = b->R;
    double U = 0.0;
    for (int a = 0; a < n; ++a) {
        int j = (a + 1) % n;
        double l = hypot(R[2 * j] - R[2 * a], R[2 * j + 1] - R[2 * a + 1]);
        U += 0.5 * b->k_spring * (l - b->l_eq) * (l - b->l_eq);
    }
    for (int a = 0; a < n; ++a) {
        int im = (a - 1 + n) % n, ip = (a + 1) % n;
        double e1x = R[2 * im] - R[2 * a], e1y = R[2 * im + 1] - R[2 * a + 1];
        double e2x = R[2 * ip] - R[2 * a], e2y = R[2 * ip + 1] - R[2 * a + 1];
        double cg = (e1x * e2x + e1y * e2y) / (hypot(e1x, e1y) * hypot(e2x, e2y));
        U += b->eps_angle * (1.0 - cos(M_PI - acos(fmax(-1.0, fmin(1.0, cg)))));
    }
    return U;
}

double orc_pull_factor(const orc_body *b, double t) {
    if (b->width <= 0.0) return 1.0;
    return 1.0 / (1.0 + exp(-(t - b->t_on) / b->width)) - 1.0 / (1.0 + exp(-(t - b->t_off) / b->width));
}

static double logistic(double x) { return 1.0 / (1.0 + exp(-x)); }
static double softplus(double x) { return x > 30.0 ? x + log1p(exp(-x)) : log1p(exp(x)); }

double orc_trap_k(const orc_body *b, double t) {
    if (b->trap_k == 0.0) return 0.0;
    return b->trap_k * (logistic((t - b->trap_t1) / b->trap_w) - logistic((t - b->trap_t2) / b->trap_w));
}

void orc_trap_pos(const orc_body *b, double t, double out[2]) {
    double w = b->trap_w, T = b->trap_t2 - b->trap_t1;
    double rho = T > 0.0 ? (w / T) * (softplus((t - b->trap_t1) / w) - softplus((t - b->trap_t2) / w)) : 0.0;
    out[0] = b->trap_x0 + b->trap_dx * rho;
    out[1] = b->trap_y0 + b->trap_dy * rho;
}

static void centre_of_mass(const orc_body *b, double c[2]) {
    c[0] = c[1] = 0.0;
    for (int a = 0; a < b->n; ++a) {
        c[0] += b->R[2 * a];
        c[1] += b->R[2 * a + 1];
    }
    c[0] /= b->n;
    c[1] /= b->n;
}

double orc_trap_energy(const orc_body *b, double t) {
    double e[2], c[2];
    orc_trap_pos(b, t, e);
    centre_of_mass(b, c);
    return 0.5 * orc_trap_k(b, t) * ((e[0] - c[0]) * (e[0] - c[0]) + (e[1] - c[1]) * (e[1] - c[1]));
}

void orc_node_forces(const orc_body *b, double t, double *f) {
    int n = b->n;
    const double *R = b->R;
    memset(f, 0, sizeof(double) * 2 * n);
    /* springs: u = k/2 (l - l_eq)^2, l = |R_{a+1} - R_a| */
    for (int a = 0; a < n; ++a) {
        int j = (a + 1) % n;
        double dx = R[2 * j] - R[2 * a], dy = R[2 * j + 1] - R[2 * a + 1];
        double l = hypot(dx, dy);
        double c = b->k_spring * (l - b->l_eq) / l;
        f[2 * a] += c * dx;
        f[2 * a + 1] += c * dy;
        f[2 * j] -= c * dx;
        f[2 * j + 1] -= c * dy;
    }
    /* bending: u = eps (1 - cos(pi - gamma)) = eps (1 + cos gamma), gamma the angle at node a
     * between e1 = R_{a-1} - R_a and e2 = R_{a+1} - R_a */
    for (int a = 0; a < n; ++a) {
        int im = (a - 1 + n) % n, ip = (a + 1) % n;
        double e1x = R[2 * im] - R[2 * a], e1y = R[2 * im + 1] - R[2 * a + 1];
        double e2x = R[2 * ip] - R[2 * a], e2y = R[2 * ip + 1] - R[2 * a + 1];
        double n1 = hypot(e1x, e1y), n2 = hypot(e2x, e2y);
        double cg = (e1x * e2x + e1y * e2y) / (n1 * n2);
        double d1x = e2x / (n1 * n2) - cg * e1x / (n1 * n1);   /* d cos(gamma) / d e1 */
        double d1y = e2y / (n1 * n2) - cg * e1y / (n1 * n1);
        double d2x = e1x / (n1 * n2) - cg * e2x / (n2 * n2);   /* d cos(gamma) / d e2 */
        double d2y = e1y / (n1 * n2) - cg * e2y / (n2 * n2);
        double e = b->eps_angle;
        f[2 * im] -= e * d1x;
        f[2 * im + 1] -= e * d1y;
        f[2 * ip] -= e * d2x;
        f[2 * ip + 1] -= e * d2y;
        f[2 * a] += e * (d1x + d2x);
        f[2 * a + 1] += e * (d1y + d2y);
    }
    double s = orc_pull_factor(b, t);
    for (int a = 0; a < n; ++a) {
        f[2 * a] += s * b->pull_fx / n;
        f[2 * a + 1] += s * b->pull_fy / n;
    }
    /* trap: -d/dR_a of k/2 |R_ext - R_com|^2 = k (R_ext - R_com) / n on every node */
    double k = orc_trap_k(b, t);
    if (k != 0.0) {
        double e[2], c[2];
        orc_trap_pos(b, t, e);
        centre_of_mass(b, c);
        for (int a = 0; a < n; ++a) {
            f[2 * a] += k * (e[0] - c[0]) / n;
            f[2 * a + 1] += k * (e[1] - c[1]) / n;
        }
    }
}

void orc_spread(const orc_params *p, int n, const double *R, const double *f, double *fx, double *fy) {
    for (int a = 0; a < n; ++a) {
        int x0 = (int)floor(R[2 * a]) - 1, y0 = (int)floor(R[2 * a + 1]) - 1;
        for (int j = 0; j < 4; ++j) {
            int y = y0 + j;
            if (p->walls && (y < 0 || y >= p->ny)) continue;
            double wy = orc_phi(R[2 * a + 1] - y);
            for (int i = 0; i < 4; ++i) {
                int x = x0 + i;
                if (p->walls == 2 && (x < 0 || x >= p->nx)) continue;
                double w = orc_phi(R[2 * a] - x) * wy;
                size_t s = (size_t)wrap(y, p->ny) * p->nx + wrap(x, p->nx);
                fx[s] += f[2 * a] * w;
                fy[s] += f[2 * a + 1] * w;
            }
        }
    }
}

void orc_interp(const orc_params *p, int n, const double *R, const double *ux, const double *uy, double *out) {
    for (int a = 0; a < n; ++a) {
        int x0 = (int)floor(R[2 * a]) - 1, y0 = (int)floor(R[2 * a + 1]) - 1;
        double vx = 0.0, vy = 0.0;
        for (int j = 0; j < 4; ++j) {
            int y = y0 + j;
            if (p->walls && (y < 0 || y >= p->ny)) continue;
            double wy = orc_phi(R[2 * a + 1] - y);
            for (int i = 0; i < 4; ++i) {
                int x = x0 + i;
                if (p->walls == 2 && (x < 0 || x >= p->nx)) continue;
                double w = orc_phi(R[2 * a] - x) * wy;
                size_t s = (size_t)wrap(y, p->ny) * p->nx + wrap(x, p->nx);
                vx += ux[s] * w;
                vy += uy[s] * w;
            }
        }
        out[2 * a] = vx;
        out[2 * a + 1] = vy;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* fluid force: f_IB + f^p + f^E + uniform g                                                   */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    size_t N;
    double *F;      /* 2N */
    double *hP;     /* 2N molecular field */
    double *sE;     /* 4N Ericksen stress: xx, xy, yx, yy */
    double *rho;    /* N */
    double *u;      /* 2N */
    double *hpost;  /* 9N */
    double *G;      /* 4N: dx vx, dx vy, dy vx, dy vy */
    double *Cst;    /* 9N stiffness */
    double *r1;     /* 3N */
    double *xs;     /* 3N predicted field */
    double *r2;     /* 3N */
    double *nodebuf;/* scratch for the nodes */
} work_t;

static void compute_force(const orc_params *p, int nb, const orc_body *bodies, const double *sigma,
                          const double *P, int t, work_t *w) {
    const int nx = p->nx, ny = p->ny;
    const size_t N = w->N;
    double *Fx = w->F, *Fy = w->F + N;
    for (size_t s = 0; s < N; ++s) { Fx[s] = p->gx; Fy[s] = p->gy; }

    /* 1-2: node forces and spreading, body by body, node by node */
    for (int b = 0; b < nb; ++b) {
        double *f = (double *)malloc(sizeof(double) * 2 * bodies[b].n);
        orc_node_forces(&bodies[b], (double)t, f);
        orc_spread(p, bodies[b].n, bodies[b].R, f, Fx, Fy);
        free(f);
    }

    /* 3: f^p_i = d_j sigma_ij */
    if (p->polymer_force) {
        const double *sxx = sigma, *syy = sigma + N, *sxy = sigma + 2 * N;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t s = (size_t)y * nx + x;
                Fx[s] += ddx(p, sxx, x, y, GHOST_EVEN) + ddy(p, sxy, x, y, GHOST_EVEN);
                Fy[s] += ddx(p, sxy, x, y, GHOST_EVEN) + ddy(p, syy, x, y, GHOST_EVEN);
            }
    }

    /* 4: molecular field, Ericksen stress, f^E_i = d_j sigmaE_ij */
    if (p->ericksen) {
        const double *Pc[2] = {P, P + N};
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t s = (size_t)y * nx + x;
                double Px = Pc[0][s], Py = Pc[1][s];
                double a = p->alpha + p->beta * (Px * Px + Py * Py);
                w->hP[s] = a * Px - p->kappa * lap5(p, Pc[0], x, y, GHOST_EVEN);
                w->hP[N + s] = a * Py - p->kappa * lap5(p, Pc[1], x, y, GHOST_EVEN);
            }
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t s = (size_t)y * nx + x;
                double Pv[2] = {Pc[0][s], Pc[1][s]};
                double hv[2] = {w->hP[s], w->hP[N + s]};
                /* dP[i][k] = d_i P_k */
                double dP[2][2] = {{ddx(p, Pc[0], x, y, GHOST_EVEN), ddx(p, Pc[1], x, y, GHOST_EVEN)},
                                   {ddy(p, Pc[0], x, y, GHOST_EVEN), ddy(p, Pc[1], x, y, GHOST_EVEN)}};
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) {
                        double v = -0.5 * (Pv[i] * hv[j] - hv[i] * Pv[j]) +
                                   0.5 * p->xi * (Pv[i] * hv[j] + hv[i] * Pv[j]) -
                                   p->kappa * (dP[i][0] * dP[j][0] + dP[i][1] * dP[j][1]);
                        w->sE[(size_t)(2 * i + j) * N + s] = v;
                    }
            }
        const double *exx = w->sE, *exy = w->sE + N, *eyx = w->sE + 2 * N, *eyy = w->sE + 3 * N;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t s = (size_t)y * nx + x;
                Fx[s] += ddx(p, exx, x, y, GHOST_EVEN) + ddy(p, exy, x, y, GHOST_EVEN);
                Fy[s] += ddx(p, eyx, x, y, GHOST_EVEN) + ddy(p, eyy, x, y, GHOST_EVEN);
            }
    }
}

/* 5: density and force-corrected velocity */
static void moments(const orc_params *p, const double *h, work_t *w) {
    const size_t N = w->N;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        double rho = 0.0, mx = 0.0, my = 0.0;
        for (int n = 0; n < 9; ++n) {
            double hn = h[(size_t)n * N + s];
            rho += hn;
            mx += CX[n] * hn;
            my += CY[n] * hn;
        }
        w->rho[s] = rho;
        w->u[s] = (mx + 0.5 * w->F[s]) / rho;
        w->u[N + s] = (my + 0.5 * w->F[N + s]) / rho;
    }
    (void)p;
}

/* 6-7: BGK + Guo source, then streaming into h */
static void collide_stream(const orc_params *p, double *h, work_t *w) {
    const int nx = p->nx, ny = p->ny;
    const size_t N = w->N;
    const double tau = p->tau;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        double rho = w->rho[s], ux = w->u[s], uy = w->u[N + s];
        double Fx = w->F[s], Fy = w->F[N + s];
        double uu = ux * ux + uy * uy;
        for (int n = 0; n < 9; ++n) {
            double cu = CX[n] * ux + CY[n] * uy;
            double heq = WQ[n] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            double S = (1.0 - 0.5 / tau) * WQ[n] *
                       (3.0 * ((CX[n] - ux) * Fx + (CY[n] - uy) * Fy) + 9.0 * cu * (CX[n] * Fx + CY[n] * Fy));
            double hn = h[(size_t)n * N + s];
            w->hpost[(size_t)n * N + s] = hn - (hn - heq) / tau + S;
        }
    }
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            for (int n = 0; n < 9; ++n) {
                /* pull form of h_n(r + c_n, t+1) = h*_n(r, t): the value arriving at (x, y) */
                int xs = x - CX[n], ys = y - CY[n];
                double v;
                if ((p->walls && (ys < 0 || ys >= ny)) || (p->walls == 2 && (xs < 0 || xs >= nx)))
                    v = w->hpost[(size_t)OPP[n] * N + s];     /* bounced back at the wall */
                else
                    v = w->hpost[(size_t)n * N + (size_t)wrap(ys, ny) * nx + wrap(xs, nx)];
                h[(size_t)n * N + s] = v;
            }
        }
}

/* 8: G = (dx vx, dx vy, dy vx, dy vy) */
static void velocity_gradient(const orc_params *p, const double *u, double *G) {
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            G[s] = ddx(p, u, x, y, GHOST_ODD);
            G[N + s] = ddx(p, u + N, x, y, GHOST_ODD);
            G[2 * N + s] = ddy(p, u, x, y, GHOST_ODD);
            G[3 * N + s] = ddy(p, u + N, x, y, GHOST_ODD);
        }
}

/* right-hand side of eqStiffCons with the corotational derivative:
 * dX/dt = -(v.grad)X - (Omega X - X Omega) + C~ Psi - C~ X / eta_p + D_p lap X */
static void rhs_sigma(const orc_params *p, const double *X, const double *u, const double *G,
                      const double *Cst, double *out) {
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    const double inv_eta = 1.0 / p->eta_p;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            double ux = u[s], uy = u[N + s];
            double om = 0.5 * (G[N + s] - G[2 * N + s]);           /* Omega_xy */
            double Psi[3] = {G[s], G[3 * N + s], 0.5 * (G[N + s] + G[2 * N + s])};
            double Xv[3] = {X[s], X[N + s], X[2 * N + s]};
            double J[3] = {2.0 * om * Xv[2], -2.0 * om * Xv[2], om * (Xv[1] - Xv[0])};
            const double *C = Cst + 9 * s;
            for (int c = 0; c < 3; ++c) {
                const double *Xc = X + (size_t)c * N;
                double adv = ux * ddx(p, Xc, x, y, GHOST_EVEN) + uy * ddy(p, Xc, x, y, GHOST_EVEN);
                double CPsi = C[3 * c] * Psi[0] + C[3 * c + 1] * Psi[1] + C[3 * c + 2] * Psi[2];
                double CX = C[3 * c] * Xv[0] + C[3 * c + 1] * Xv[1] + C[3 * c + 2] * Xv[2];
                out[(size_t)c * N + s] = -adv - J[c] + CPsi - CX * inv_eta + p->D_p * lap5(p, Xc, x, y, GHOST_EVEN);
            }
        }
}

/* right-hand side of eqBE:  dY/dt = -(v.grad)Y - Omega Y + xi Psi Y - Gamma h(Y) */
static void rhs_P(const orc_params *p, const double *Y, const double *u, const double *G, double *out) {
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            double ux = u[s], uy = u[N + s];
            double om = 0.5 * (G[N + s] - G[2 * N + s]);
            double Pxx = G[s], Pyy = G[3 * N + s], Pxy = 0.5 * (G[N + s] + G[2 * N + s]);
            double Yx = Y[s], Yy = Y[N + s];
            double a = p->alpha + p->beta * (Yx * Yx + Yy * Yy);
            double hx = a * Yx - p->kappa * lap5(p, Y, x, y, GHOST_EVEN);
            double hy = a * Yy - p->kappa * lap5(p, Y + N, x, y, GHOST_EVEN);
            double advx = ux * ddx(p, Y, x, y, GHOST_EVEN) + uy * ddy(p, Y, x, y, GHOST_EVEN);
            double advy = ux * ddx(p, Y + N, x, y, GHOST_EVEN) + uy * ddy(p, Y + N, x, y, GHOST_EVEN);
            out[s] = -advx - om * Yy + p->xi * (Pxx * Yx + Pxy * Yy) - p->Gamma * hx;
            out[N + s] = -advy + om * Yx + p->xi * (Pxy * Yx + Pyy * Yy) - p->Gamma * hy;
        }
}

static void alloc_work(work_t *w, size_t N, int nb, const orc_body *bodies) {
    int maxn = 1;
    for (int b = 0; b < nb; ++b) if (bodies[b].n > maxn) maxn = bodies[b].n;
    w->N = N;
    w->F = (double *)calloc(2 * N, sizeof(double));
    w->hP = (double *)calloc(2 * N, sizeof(double));
    w->sE = (double *)calloc(4 * N, sizeof(double));
    w->rho = (double *)calloc(N, sizeof(double));
    w->u = (double *)calloc(2 * N, sizeof(double));
    w->hpost = (double *)calloc(9 * N, sizeof(double));
    w->G = (double *)calloc(4 * N, sizeof(double));
    w->Cst = (double *)calloc(9 * N, sizeof(double));
    w->r1 = (double *)calloc(3 * N, sizeof(double));
    w->xs = (double *)calloc(3 * N, sizeof(double));
    w->r2 = (double *)calloc(3 * N, sizeof(double));
    w->nodebuf = (double *)calloc(8 * (size_t)maxn, sizeof(double));
}

static void free_work(work_t *w) {
    free(w->F); free(w->hP); free(w->sE); free(w->rho); free(w->u); free(w->hpost);
    free(w->G); free(w->Cst); free(w->r1); free(w->xs); free(w->r2); free(w->nodebuf);
}

void orc_run(const orc_params *p, int nb, orc_body *bodies, double *h, double *sigma, double *P,
             const double *u_kin, int t0, int n_steps) {
    const size_t N = (size_t)p->nx * p->ny;
    work_t w;
    alloc_work(&w, N, nb, bodies);
    for (int step = 0; step < n_steps; ++step) {
        /* fluid: forces at t, moments at t, then h -> h(t+1) */
        if (p->kinematic) {
            memcpy(w.u, u_kin, sizeof(double) * 2 * N);
        } else {
            compute_force(p, nb, bodies, sigma, P, t0 + step, &w);
            moments(p, h, &w);
            collide_stream(p, h, &w);
        }
        /* velocity gradient of v(t) */
        velocity_gradient(p, w.u, w.G);
        /* stiffness from P(t) */
        if (p->evolve_sigma) {
#pragma omp parallel for num_threads(g_threads) schedule(static)
            for (long long s = 0; s < (long long)N; ++s)
                orc_stiffness(P[s], P[N + s], p->Kx, p->P_clamp, w.Cst + 9 * s);
            /* Heun: X* = X + R(X); X' = X + (R(X) + R(X*))/2 */
            rhs_sigma(p, sigma, w.u, w.G, w.Cst, w.r1);
            for (size_t i = 0; i < 3 * N; ++i) w.xs[i] = sigma[i] + w.r1[i];
            rhs_sigma(p, w.xs, w.u, w.G, w.Cst, w.r2);
            for (size_t i = 0; i < 3 * N; ++i) sigma[i] += 0.5 * (w.r1[i] + w.r2[i]);
        }
        if (p->evolve_P) {
            rhs_P(p, P, w.u, w.G, w.r1);
            for (size_t i = 0; i < 2 * N; ++i) w.xs[i] = P[i] + w.r1[i];
            rhs_P(p, w.xs, w.u, w.G, w.r2);
            for (size_t i = 0; i < 2 * N; ++i) P[i] += 0.5 * (w.r1[i] + w.r2[i]);
        }
        /* nodes: R* = R + v(R); R' = R + (v(R) + v(R*))/2 with the fluid velocity of time t */
        for (int b = 0; b < nb; ++b) {
            int n = bodies[b].n;
            double *R = bodies[b].R;
            double *v1 = w.nodebuf, *Rs = w.nodebuf + 2 * n, *v2 = w.nodebuf + 4 * n;
            orc_interp(p, n, R, w.u, w.u + N, v1);
            for (int i = 0; i < 2 * n; ++i) Rs[i] = R[i] + v1[i];
            orc_interp(p, n, Rs, w.u, w.u + N, v2);
            for (int i = 0; i < 2 * n; ++i) R[i] += 0.5 * (v1[i] + v2[i]);
        }
    }
    free_work(&w);
}

void orc_observe(const orc_params *p, int nb, const orc_body *bodies, const double *h,
                 const double *sigma, const double *P, const double *u_kin, int t, double *out) {
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    work_t w;
    alloc_work(&w, N, nb, bodies);
    if (p->kinematic) {
        memcpy(w.u, u_kin, sizeof(double) * 2 * N);
        for (size_t s = 0; s < N; ++s) { w.rho[s] = 1.0; w.F[s] = 0.0; w.F[N + s] = 0.0; }
    } else {
        compute_force(p, nb, bodies, sigma, P, t, &w);
        moments(p, h, &w);
    }
    for (size_t s = 0; s < N; ++s) {
        out[s] = w.rho[s];
        out[N + s] = w.u[s];
        out[2 * N + s] = w.u[N + s];
        out[5 * N + s] = w.F[s];
        out[6 * N + s] = w.F[N + s];
    }
    const double *sxx = sigma, *syy = sigma + N, *sxy = sigma + 2 * N;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            out[3 * N + s] = ddx(p, sxx, x, y, GHOST_EVEN) + ddy(p, sxy, x, y, GHOST_EVEN);
            out[4 * N + s] = ddx(p, sxy, x, y, GHOST_EVEN) + ddy(p, syy, x, y, GHOST_EVEN);
        }
    free_work(&w);
}

/* even-odd crossing test, half-open in y */
static int inside_polygon(int n, const double *R, double px, double py) {
    int in = 0;
    for (int i = 0, j = n - 1; i < n; j = i++) {
        double xi = R[2 * i], yi = R[2 * i + 1], xj = R[2 * j], yj = R[2 * j + 1];
        if ((yi > py) != (yj > py) && px < (xj - xi) * (py - yi) / (yj - yi) + xi) in = !in;
    }
    return in;
}

void orc_body_force(const orc_params *p, const orc_body *b, const double *sigma, double *out) {
    const int nx = p->nx;
    const size_t N = (size_t)nx * p->ny;
    const double *sxx = sigma, *syy = sigma + N, *sxy = sigma + 2 * N;
    double minx = b->R[0], maxx = b->R[0], miny = b->R[1], maxy = b->R[1], cx = 0.0, cy = 0.0;
    for (int a = 0; a < b->n; ++a) {
        double x = b->R[2 * a], y = b->R[2 * a + 1];
        minx = fmin(minx, x); maxx = fmax(maxx, x);
        miny = fmin(miny, y); maxy = fmax(maxy, y);
        cx += x; cy += y;
    }
    double fx = 0.0, fy = 0.0;
    for (int y = (int)ceil(miny); y <= (int)floor(maxy); ++y)
        for (int x = (int)ceil(minx); x <= (int)floor(maxx); ++x) {
            if (!inside_polygon(b->n, b->R, x, y)) continue;
            fx += ddx(p, sxx, x, y, GHOST_EVEN) + ddy(p, sxy, x, y, GHOST_EVEN);
            fy += ddx(p, sxy, x, y, GHOST_EVEN) + ddy(p, syy, x, y, GHOST_EVEN);
        }
    out[0] = fx;
    out[1] = fy;
    out[2] = cx / b->n;
    out[3] = cy / b->n;
}

/* ------------------------------------------------------------------------------------------ */
/* area-weighted restoring force                                                               */
/* ------------------------------------------------------------------------------------------ */

/* Clip a polygon against one half-plane (Sutherland-Hodgman): keep points with
 * side * (coordinate axis of q - c) >= 0.  Returns the new vertex count. */
static int clip_half(const double *in, int n, double *out, int axis, double c, double side) {
    int m = 0;
    for (int i = 0; i < n; ++i) {
        const double *a = in + 2 * ((i + n - 1) % n), *b = in + 2 * i;
        double da = side * (a[axis] - c), db = side * (b[axis] - c);
        if (db >= 0.0) {
            if (da < 0.0) {
                double t = da / (da - db);
                out[2 * m] = a[0] + t * (b[0] - a[0]);
                out[2 * m + 1] = a[1] + t * (b[1] - a[1]);
                out[2 * m + axis] = c;
                ++m;
            }
            out[2 * m] = b[0];
            out[2 * m + 1] = b[1];
            ++m;
        } else if (da >= 0.0) {
            double t = da / (da - db);
            out[2 * m] = a[0] + t * (b[0] - a[0]);
            out[2 * m + 1] = a[1] + t * (b[1] - a[1]);
            out[2 * m + axis] = c;
            ++m;
        }
    }
    return m;
}

static double shoelace(const double *q, int n) {
    double a = 0.0;
    for (int i = 0, j = n - 1; i < n; j = i++) a += q[2 * j] * q[2 * i + 1] - q[2 * i] * q[2 * j + 1];
    return 0.5 * a;
}

double orc_cell_area(int n, const double *R, double x0, double x1, double y0, double y1) {
    double *A = malloc(sizeof(double) * 2 * (n + 8)), *B = malloc(sizeof(double) * 2 * (n + 8));
    int m = n;
    memcpy(A, R, sizeof(double) * 2 * n);
    m = clip_half(A, m, B, 0, x0, 1.0);
    m = clip_half(B, m, A, 0, x1, -1.0);
    m = clip_half(A, m, B, 1, y0, 1.0);
    m = clip_half(B, m, A, 1, y1, -1.0);
    double area = m >= 3 ? shoelace(A, m) : 0.0;
    free(A);
    free(B);
    return shoelace(R, n) < 0.0 ? -area : area;
}

void orc_body_force_area(const orc_params *p, const orc_body *b, const double *sigma, double *out) {
    const size_t N = (size_t)p->nx * p->ny;
    const double *sxx = sigma, *syy = sigma + N, *sxy = sigma + 2 * N;
    double minx = b->R[0], maxx = b->R[0], miny = b->R[1], maxy = b->R[1];
    for (int a = 0; a < b->n; ++a) {
        minx = fmin(minx, b->R[2 * a]); maxx = fmax(maxx, b->R[2 * a]);
        miny = fmin(miny, b->R[2 * a + 1]); maxy = fmax(maxy, b->R[2 * a + 1]);
    }
    double fx = 0.0, fy = 0.0;
    for (int y = (int)floor(miny + 0.5); y <= (int)ceil(maxy - 0.5); ++y)
        for (int x = (int)floor(minx + 0.5); x <= (int)ceil(maxx - 0.5); ++x) {
            double w = orc_cell_area(b->n, b->R, x - 0.5, x + 0.5, y - 0.5, y + 0.5);
            if (w == 0.0) continue;
            fx += w * (ddx(p, sxx, x, y, GHOST_EVEN) + ddy(p, sxy, x, y, GHOST_EVEN));
            fy += w * (ddx(p, sxy, x, y, GHOST_EVEN) + ddy(p, syy, x, y, GHOST_EVEN));
        }
    out[0] = fx;
    out[1] = fy;
}
