/*
 * Plain FP64 CPU oracle for the viscoelastic immersed-boundary lattice Boltzmann step
 * (Floyd, Vaikuntanathan, Dinner, "Simulating structured fluids with tensorial
 * viscoelasticity", arXiv 2209.14889).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source, header, table or helper with the
 * GPU library and the library never calls it.
 *
 * Conventions (lattice units, dx = dt = 1, rho0 = 1, cs^2 = 1/3):
 *   - fields are planes of ny*nx doubles, x fastest: f[y*nx + x];
 *   - populations h are stored as full values (not offsets), 9 planes, pre-collision at time t;
 *   - sigma = (sxx, syy, sxy) planes; P = (Px, Py) planes;
 *   - body node positions are unwrapped lattice coordinates, interleaved x0,y0,x1,y1,...
 */
#ifndef VELB_ORACLE_H
#define VELB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny;
    int walls;          /* 0: periodic in x and y; 1: halfway bounce-back walls at y=-1/2 and y=ny-1/2;
                           2: a closed box, walls also at x=-1/2 and x=nx-1/2 */
    double tau;         /* BGK relaxation time */
    double Kx[4];       /* K1111, K1122, K2222, K1212 of the aligned stiffness tensor */
    double eta_p;       /* polymer viscosity; +inf switches the relaxation term off */
    double D_p;         /* stress diffusion constant */
    double xi, alpha, beta, kappa, Gamma;   /* Beris-Edwards / free-energy coefficients */
    double P_clamp;     /* magnitude cap used only when inverting P(k) */
    int ericksen;       /* 1: Ericksen force enters the fluid force */
    int polymer_force;  /* 1: divergence of the polymer stress enters the fluid force */
    int evolve_sigma;   /* 1: integrate the polymer stress */
    int evolve_P;       /* 1: integrate the polarization */
    int kinematic;      /* 1: the fluid is not evolved; the velocity is the prescribed field u_kin */
    double gx, gy;      /* uniform body-force density added everywhere */
} orc_params;

typedef struct {
    int n;              /* number of nodes on the closed loop */
    double k_spring, eps_angle, l_eq;
    double pull_fx, pull_fy;  /* total external force, shared equally by the nodes */
    double t_on, t_off, width;/* pull switched on/off by logistic functions of time (steps) of
                                 scale `width` centred at t_on and t_off; width <= 0: constant */
    /* harmonic trap on the centre of mass (App. A, eqUtrap): u = k(t)/2 |R_ext(t) - R_com|^2 with
     * k(t) = trap_k [S((t - t1)/w) - S((t - t2)/w)], S the logistic function, and
     * R_ext(t) = (trap_x0, trap_y0) + (trap_dx, trap_dy) rho(t), where
     * rho(t) = (w / (t2 - t1)) [sp((t - t1)/w) - sp((t - t2)/w)], sp(x) = ln(1 + e^x): the trap
     * moves at constant speed from t1 to t2 with logistic starts and stops (the integral of the
     * switching function) and lets go at t2.  trap_k = 0: no trap. */
    double trap_k, trap_x0, trap_y0, trap_dx, trap_dy, trap_t1, trap_t2, trap_w;
    double *R;          /* 2n doubles, updated in place */
} orc_body;

/* threads used by the site loops (OpenMP); results do not depend on it */
void orc_set_threads(int n);
int orc_get_threads(void);

/* modified Bessel function of the first kind, integer order n >= 0, by its power series */
double orc_bessel_i(int n, double k);
/* inverse of P(k) = I1(k)/I0(k) on [0, 1) */
double orc_k_of_p(double p);
/* plain-component 3x3 stiffness operator C~(P), row-major, acting on (Xxx, Xyy, Xxy) */
void orc_stiffness(double Px, double Py, const double Kx[4], double P_clamp, double C[9]);

/* cosine 4-point immersed-boundary kernel */
double orc_phi(double r);
/* pull schedule factor at time t (1 when width <= 0) */
double orc_pull_factor(const orc_body *b, double t);
/* node forces -dU/dR (spring + bending + trap) plus the pull share at time t; f has 2n entries */
void orc_node_forces(const orc_body *b, double t, double *f);
/* total elastic energy of the loop (spring + bending), pull and trap excluded */
double orc_body_energy(const orc_body *b);
/* trap stiffness k(t), trap position R_ext(t) (out[2]) and trap energy at time t */
double orc_trap_k(const orc_body *b, double t);
void orc_trap_pos(const orc_body *b, double t, double out[2]);
double orc_trap_energy(const orc_body *b, double t);
/* add sum_a f_a phi phi to the force planes fx, fy (ny*nx each) */
void orc_spread(const orc_params *p, int n, const double *R, const double *f, double *fx, double *fy);
/* interpolate the velocity planes ux, uy at n points R -> out (2n) */
void orc_interp(const orc_params *p, int n, const double *R, const double *ux, const double *uy, double *out);

/* advance n_steps coupled steps; every state array is updated in place.
 * h: 9 planes, sigma: 3 planes, P: 2 planes, u_kin: 2 planes (read only when kinematic). */
void orc_run(const orc_params *p, int n_bodies, orc_body *bodies,
             double *h, double *sigma, double *P, const double *u_kin, int t0, int n_steps);

/* observables at the current time t (before the next update), planes of ny*nx:
 * out = [rho, vx, vy, fpx, fpy, Fx, Fy]   (7 planes)
 * v is the force-corrected velocity, fp = div sigma, F = total fluid force. */
void orc_observe(const orc_params *p, int n_bodies, const orc_body *bodies,
                 const double *h, const double *sigma, const double *P, const double *u_kin,
                 int t, double *out);

/* restoring force of a body: sum of div(sigma) over the lattice sites strictly inside its
 * node polygon (even-odd rule), in out[0..1]; out[2..3] = centre of mass of the nodes */
void orc_body_force(const orc_params *p, const orc_body *b, const double *sigma, double *out);

/* area of (node polygon) intersected with the box [x0, x1] x [y0, y1], by clipping the polygon
 * against the box's four half-planes and taking the shoelace area; positive for either
 * orientation of a simple polygon */
double orc_cell_area(int n, const double *R, double x0, double x1, double y0, double y1);

/* area-weighted restoring force: the integral of div(sigma) over the body with div(sigma) taken
 * constant on each lattice cell [x-1/2, x+1/2] x [y-1/2, y+1/2], i.e. the sum over sites of
 * (cell area inside the polygon) * div(sigma); out[0..1].  Unlike the site sum above it varies
 * continuously with the node positions. */
void orc_body_force_area(const orc_params *p, const orc_body *b, const double *sigma, double *out);

#ifdef __cplusplus
}
#endif
#endif
