/*
 * liblb: MI355X (gfx950) library for the coupled viscoelastic immersed-boundary lattice
 * Boltzmann step of Floyd, Vaikuntanathan and Dinner, "Simulating structured fluids with
 * tensorial viscoelasticity" (arXiv 2209.14889).
 *
 * The problem (abstract, Sec. II): an elastic body immersed in a structured fluid is driven by an
 * external force.  The state is {h_n (fluid populations), sigma^p (polymer stress), P
 * (polarization), R_a (body nodes)} (Fig. 2).  One step updates every field from the previous
 * time step: D2Q9 BGK collide-stream with Guo forcing by F = f_IB + div sigma^p + div sigma^E
 * (Sec. II A-C, App. A), Heun predictor-corrector for sigma^p (eqStiffCons, corotational) and P
 * (eqBE), and overdamped no-slip node motion (App. A).
 *
 * Conventions for every entry point:
 *   - return 0 (LB_OK) on success or a negative LB_E* code; lb_last_error() then holds a message
 *     for the calling thread;
 *   - lattice units (dx = dt = 1); fields are planes of ny*nx values with x fastest;
 *   - host pointers are read during the call only and are never retained; device memory is the
 *     caller-owned arena passed to lb_create, which the library never frees;
 *   - a handle is bound to one HIP stream and is not thread safe; lb_step is asynchronous, and
 *     faults of its kernels (LB_EDEVICE) or a raised watchdog (LB_EUNSTABLE) are reported by the
 *     next synchronising call (lb_read_fields, lb_body_force, lb_conservation, lb_sync) and by
 *     later lb_step calls;
 *   - no C++ exception crosses the boundary; null pointers are rejected with LB_EINVAL.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_EINVAL (-1)     /* invalid argument or parameter (see lb_create) */
#define LB_ENOMEM (-2)     /* arena too small */
#define LB_EDEVICE (-3)    /* HIP runtime error */
#define LB_EUNSTABLE (-4)  /* watchdog: non-finite or drifting mass */
#define LB_ERANGE (-5)     /* index out of range, or a body outgrew its force patch */

typedef struct lb_handle lb_handle;

/* One immersed elastic body (App. A): a closed loop of n_nodes points with springs
 * k_spring/2 (l_a - l_eq)^2 and bending eps_angle (1 - cos(pi - gamma_a)).  The external drive
 * is a total force (pull_fx, pull_fy) shared equally by the nodes, optionally switched on and
 * off by logistic functions of time (App. C: sigmoid protocol) of scale pull_width steps centred
 * at pull_t_on and pull_t_off; pull_width <= 0 means a constant pull. */
typedef struct {
    double cx, cy, radius;      /* regular polygon, node a at angle 2 pi a / n_nodes */
    int32_t n_nodes;            /* 3 .. 1024 */
    double k_spring, eps_angle, l_eq;
    double pull_fx, pull_fy;    /* constant total pull, shared equally by the nodes, switched on and
                                   off by logistics of scale pull_width (<= 0: always on) centred
                                   at pull_t_on and pull_t_off (steps) */
    double pull_t_on, pull_t_off, pull_width;
    /* harmonic trap on the centre of mass (App. A, eqUtrap), trap_k = 0: none.  Stiffness
     * k(t) = trap_k [S((t - t1)/w) - S((t - t2)/w)] with S the logistic function; position
     * R_ext(t) = (trap_x0, trap_y0) + (trap_dx, trap_dy) rho(t) with
     * rho(t) = w / (t2 - t1) [sp((t - t1)/w) - sp((t - t2)/w)], sp(x) = ln(1 + e^x): the trap
     * moves the distance (trap_dx, trap_dy) at constant speed between t1 and t2 with logistic
     * starts and stops, and lets go at t2.  Each node gets k(t) (R_ext - R_com) / n_nodes. */
    double trap_k, trap_x0, trap_y0, trap_dx, trap_dy, trap_t1, trap_t2, trap_w;
    const double *nodes;        /* optional host array of 2*n_nodes unwrapped positions
                                   (x0, y0, x1, y1, ...) replacing the polygon; may be NULL */
} lb_body_desc;

/* One simulation on an nx x ny lattice, periodic or bounded by walls (see `walls`). */
typedef struct {
    int32_t nx, ny;             /* 8 .. 16384 each, nx*ny <= 1e8 */
    double tau;                 /* BGK relaxation time (eqBGK), > 0.5 */
    double Kx[4];               /* K1111, K1122, K2222, K1212 of the aligned stiffness (eqKmatrix) */
    double eta_p;               /* polymer viscosity (eqStiffCons), > 0 (may be +inf) */
    double D_p;                 /* stress diffusion, 0 <= D_p < 0.25 (Heun stability) */
    double xi, alpha, beta, kappa, Gamma;  /* Beris-Edwards and free energy (eqBE, eqFfunctional) */
    double P_clamp;             /* magnitude cap when inverting P(k) (eqPk), in (0, 1) */
    int32_t ericksen;           /* 1: the Ericksen force enters F (the paper's model) */
    int32_t walls;              /* 0: periodic; 1: walls half a site below row 0 and above row ny-1,
                                   x periodic (a channel); 2: also half a site left of column 0 and
                                   right of column nx-1 (a closed box, the paper's geometry).  At a
                                   wall (App. C): halfway bounce-back of the populations, mirror
                                   ghosts for sigma, P and the Ericksen stress, odd (no-slip) ghosts
                                   for the velocity gradient.  Every node's 4x4 kernel footprint
                                   must stay inside the walls with one site to spare (LB_EINVAL in
                                   lb_create, LB_ERANGE later) */
    double gx, gy;              /* uniform body force density added to F at every site */
    int32_t n_bodies;           /* 0 .. 64 */
    const lb_body_desc *bodies;
    const double *init_P;       /* host 2*nx*ny (Px plane, Py plane) or NULL (P = 0) */
    const double *init_sigma;   /* host 3*nx*ny (sxx, syy, sxy) or NULL (sigma = 0) */
    const double *init_h;       /* host 9*nx*ny pre-collision populations h_n (eqLB: after streaming,
                                   before the next collision; plane n = direction n) or NULL (the
                                   rest state); with init_sigma, init_P and explicit node positions
                                   it restarts a saved state */
} lb_sim_params;

typedef struct {
    int32_t precision;          /* 0: FP32 populations stored as offsets from the rest weights;
                                   1: FP16 storage of those offsets times 2^fp16_shift (FP32 math) */
    int32_t fp16_shift;         /* 0 selects the default 10 */
    int32_t watchdog_every;     /* FP64 mass / finiteness check every this many steps; 0 = off */
    int32_t graph_chunk;        /* steps captured per hipGraph (even); 0 = plain launches */
    int32_t kernel;             /* 0: fused single-pass field kernel; 1: multi-pass kernels */
    int32_t timing;             /* 1: time every field-kernel launch with HIP events */
    int32_t seg_rows;           /* rows per fused work item; 0 = tuned default */
    int32_t fused_threads;      /* fused work-group size: 64, 128 or 256 (strip of 56, 120 or 248
                                   columns); 0 = chosen from the lattice width */
    int32_t autotune;           /* 1: time candidate (work-group size, rows per item, grid) shapes on
                                   the live state in lb_create and keep the fastest; 0: cost model */
    int32_t grid;               /* fused work-groups launched: 0 = one per work item; > 0 = a
                                   persistent grid of that many looping over the items */
    const char *autotune_cache; /* with autotune = 1: path of a text file of tuned launch shapes,
                                   one line per key (the simulations' sizes and walls, P or not,
                                   precision, field kernel, fused_threads and the GPU model); a key
                                   found there is used without timing, a new one is tuned and its
                                   shape appended.  NULL: no file.  A missing, unreadable or
                                   garbled file only means tuning again */
} lb_options;

/* Bytes of device memory lb_create needs for these simulations (arena for all state, tables,
 * patches and scratch).  sims: n_sims parameter sets; opt may be NULL (defaults). */
int lb_query_arena_bytes(const lb_sim_params *sims, int32_t n_sims, const lb_options *opt,
                         size_t *bytes);

/* Create a handle for n_sims independent simulations advanced together (n_sims > 1 is the
 * batched ensemble; sizes may differ).  device_arena: caller-owned device memory of at least
 * lb_query_arena_bytes bytes, 256-byte aligned.  hip_stream: the stream (hipStream_t) all work
 * is issued on; NULL makes the library create its own.  Validates: tau > 0.5, 8 D_p < 2,
 * 0 < P_clamp < 1, eta_p > 0, sizes, node counts, that every body's force patch fits the
 * lattice and that no two bodies' bounding circles (centre of the nodes, farthest node)
 * intersect, across periodic directions too (LB_EINVAL otherwise, also for an arena not 256-byte aligned; LB_ENOMEM if arena_bytes
 * is smaller than lb_query_arena_bytes).  Uploads the initial state and spreads the initial body
 * forces; synchronous. */
int lb_create(const lb_sim_params *sims, int32_t n_sims, const lb_options *opt,
              void *device_arena, size_t arena_bytes, void *hip_stream, lb_handle **out);

/* Advance every simulation by n_steps >= 0 coupled steps (asynchronous on the stream; LB_EINVAL
 * for n_steps < 0).  A watchdog or patch report from earlier steps that has completed by the
 * call is returned here (LB_EUNSTABLE, LB_ERANGE) before any new work is queued. */
int lb_step(lb_handle *h, int32_t n_steps);

/* Field selection bits for lb_read_fields, in output order. */
#define LB_F_RHO   (1u << 0)   /* density, sum h (eqrhoDef) */
#define LB_F_VX    (1u << 1)   /* velocity (sum c h + F/2)/rho (eqvDef with Guo's half force) */
#define LB_F_VY    (1u << 2)
#define LB_F_SXX   (1u << 3)   /* polymer stress */
#define LB_F_SYY   (1u << 4)
#define LB_F_SXY   (1u << 5)
#define LB_F_PX    (1u << 6)   /* polarization */
#define LB_F_PY    (1u << 7)
#define LB_F_FPX   (1u << 8)   /* restoring force density div sigma^p (Figs. 5, 6, 10) */
#define LB_F_FPY   (1u << 9)
#define LB_F_NODES (1u << 10)  /* all bodies' node positions, 2 per node, body by body */
#define LB_F_ALL   0x7FFu

/* Read the selected fields of simulation `sim` at the current time into host_out (FP64):
 * each selected plane is ny*nx values, planes in bit order, then the nodes if selected.
 * n_out is the capacity of host_out in doubles (LB_ERANGE if too small).  Synchronous. */
int lb_read_fields(lb_handle *h, int32_t sim, uint32_t field_mask, double *host_out, size_t n_out);

/* Body observables at the current time, FP64 (synchronous):
 * out[0..1] restoring force: sum of div sigma^p over the lattice sites inside the node polygon;
 * out[2..3] the current external force (pull plus trap); out[4..5] centre of mass of the nodes;
 * out[6..7] total force the nodes apply to the fluid (sum_a f_a). */
int lb_body_force(lb_handle *h, int32_t sim, int32_t body, double out[8]);

/* lb_body_force for every body of every simulation at once (simulations in order, bodies in
 * order within each): 10 doubles per body into host_out (capacity n_out doubles, LB_ERANGE if
 * smaller than 10 * total bodies): the 8 values of lb_body_force, then [8..9] the area-weighted
 * restoring force, the sum over sites of (area of the site's unit cell [x-1/2, x+1/2] x
 * [y-1/2, y+1/2] inside the node polygon) * div sigma^p, which unlike out[0..1] varies
 * continuously as the body moves (the same integral over the body, Sec. III and Fig. 6, with a
 * different quadrature).  Synchronous. */
int lb_body_forces(lb_handle *h, double *host_out, size_t n_out);

/* lb_body_forces without synchronising, for sampling a run on the device: queues the observable
 * kernel on the handle's stream and writes 8 doubles per body (simulations in order, bodies in
 * order within each) into device_out, device memory of at least n_out doubles (LB_ERANGE if
 * n_out < 8 * total bodies): [0..1] the site-sum restoring force, [2..3] the centre of mass,
 * [4..5] the total node force, [6..7] the area-weighted restoring force (the same quantities as
 * lb_body_forces, without the external force, which the host computes).  Asynchronous. */
int lb_body_forces_device(lb_handle *h, double *device_out, size_t n_out);

/* Bytes of stored state one site update reads and writes (populations, polymer stress and
 * polarization planes, read once and written once) in this handle's storage form. */
int lb_state_bytes(lb_handle *h, double *bytes_per_site);

/* Copy `bytes` of device memory from src to dst on hip_stream (NULL: the null stream) with the
 * library's streaming copy kernel: the bandwidth ceiling the field kernel is measured against.
 * bytes and both pointers must be multiples of 16 (LB_EINVAL otherwise); the buffers must not
 * overlap.  Asynchronous. */
int lb_stream_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

/* FP64 conservation sums of simulation `sim` at the current time (synchronous):
 * out[0] = sum rho, out[1..2] = sum of sum_n c_n h_n (momentum without the half force). */
int lb_conservation(lb_handle *h, int32_t sim, double out[3]);

/* Wait for all queued work; reports deferred device errors and the watchdog. */
int lb_sync(lb_handle *h);

/* Steps taken so far. */
int lb_time(lb_handle *h, int64_t *t);

/* With opt.timing = 1: total milliseconds and number of field-kernel launches timed so far, and
 * the same for the immersed-boundary kernel; counters reset when reset != 0.  Synchronous. */
int lb_timing(lb_handle *h, double *field_ms, int64_t *field_launches, double *ib_ms,
              int64_t *ib_launches, int32_t reset);

/* Fused-kernel launch shape in use: work-group size, rows per work item, number of work items,
 * work-groups launched (fewer than the items: a persistent grid looping over them), and (after
 * autotuning) the measured milliseconds per launch of the chosen shape (else 0).  Any output
 * pointer may be NULL. */
int lb_launch_shape(lb_handle *h, int32_t *threads, int32_t *seg_rows, int32_t *n_items, int32_t *grid,
                    double *tuned_ms);

/* Release the handle's host resources (and its stream if the library created it). */
int lb_destroy(lb_handle *h);

/* Message of the last failure on this thread ("" if none). */
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
