/*
 * lbddf.h - C ABI of the MI355X (gfx950) implementation of the coupled
 * double-distribution-function thermal lattice Boltzmann model on D2Q9
 * (Li, Luo, He, Gao & Tao, "Coupling lattice Boltzmann model for simulation of
 * thermal flows on standard lattices").
 *
 * One time step advances the density populations f^ (MRT collision, Eq. 44,
 * or BGK, Eq. 34) and the energy populations h- (BGK with the viscous-heating
 * coupling term, Eq. 47, or Eq. 38 without it) with the theta-coupled
 * equilibria of Eq. 18 / Eq. 41, the D2Q9 correction term of Eq. 48-50 and the
 * forcing term of Eq. 51, then streams them (Eq. 45).  Macroscopic values are
 * recovered by Eq. 46, the forcing note after Eq. 51 and Eq. 37 (or the
 * internal-energy form of Sec. III-C-1).
 *
 * Units: lattice units, dx = dt = c = 1, so R * T0 must equal 1/3 (Sec. II,
 * Sec. IV-A); lb_create rejects other values.
 *
 * Arithmetic: liblbddf.so computes the step in FP32; on grids with walls and
 * FP32 storage it forms the moment sums, the non-equilibrium parts m - m_eq
 * and h - h_eq and the wall rebuild in FP64 and applies the increments in
 * FP32 (the long gravity-driven cavity runs need it).  liblbddf_fp64.so, built
 * from the same source, exports the same ABI with the step's arithmetic in
 * FP64 and the same storage formats and state layout; its FP32 stores round
 * stochastically (about half the throughput; for flows whose FP32 rounding
 * of large deviations from rest, such as a gravity-stratified cavity,
 * exceeds what a result can tolerate).  A state created by one library must
 * be stepped by the same one.
 *
 * Memory: the caller owns one device buffer of lb_state_bytes() bytes
 * (256-byte aligned) and keeps it alive until lb_destroy.  The library
 * allocates no device memory; it keeps host-side state, the hipGraph of its
 * step batches, and one static 64 KiB device array per GPU that
 * lb_diag_noalloc uses for partial sums.  All device work
 * runs asynchronously on the HIP stream given to lb_create (NULL: the null
 * stream); calls that return data to host memory synchronise that stream.
 *
 * Errors: every call returns an lb_status; nothing throws across the ABI.
 * lb_last_error() returns the message of the last failure on the calling
 * thread.  One handle must not be used by two threads at once.
 *
 * Field arrays on the host are row-major [ny][nx] doubles (x fastest);
 * population arrays are [18][ny][nx], f^ in planes 0..8 and h- in 9..17, in the
 * velocity order of Eq. 6: e0 = (0,0), e1..e4 = (1,0),(0,1),(-1,0),(0,-1),
 * e5..e8 = (1,1),(-1,1),(-1,-1),(1,-1).
 */
#ifndef LBDDF_H
#define LBDDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,    /* invalid argument or parameter set */
    LB_ENOMEM = -2,    /* the caller's buffer is smaller than lb_state_bytes() */
    LB_EHIP = -3,      /* a HIP runtime call failed */
    LB_EUNSTABLE = -4, /* a node holds a non-finite value, rho <= 0 or T <= 0 */
    LB_EBUSY = -5      /* the serving queue is full */
} lb_status;

typedef enum { LB_STORE_F32 = 0, LB_STORE_F16 = 1, LB_STORE_BF16 = 2 } lb_storage;
typedef enum { LB_ENERGY_TOTAL = 0, LB_ENERGY_INTERNAL = 1 } lb_energy;
typedef enum { LB_VISC_CONST_TAU = 0, LB_VISC_CONST_MU = 1, LB_VISC_POWER = 2, LB_VISC_SUTHERLAND = 3 } lb_visc;
typedef enum { LB_BC_PERIODIC = 0, LB_BC_WALL = 1, LB_BC_ADIABATIC = 2, LB_BC_INLET = 3, LB_BC_OUTLET = 4 } lb_bc_kind;
typedef enum { LB_COLLIDE_MRT = 0, LB_COLLIDE_BGK = 1 } lb_collision;
typedef enum { LB_RHO_PRESSURE = 0, LB_RHO_DENSITY = 1 } lb_rho_extrap;

/* One side of the domain (x-, x+, y-, y+ in that order).  Walls sit on the
 * outermost nodes and use non-equilibrium extrapolation from the nearest
 * interior node (Sec. IV-A, IV-C):
 *   LB_BC_WALL       velocity (ux, uy) and temperature T prescribed;
 *   LB_BC_ADIABATIC  velocity prescribed, zero normal temperature gradient
 *                    (second-order one-sided: T_b = (4 T_1 - T_2) / 3);
 *   LB_BC_INLET      x- only: post-collision populations reset every step to
 *                    the equilibria at u = amp s, rho = rho0 (1 + amp s / c_s),
 *                    T = T0 (1 + (gamma - 1) amp s / c_s), s = sin(2 pi n / period),
 *                    c_s = sqrt(gamma R T0) (Eq. 53-54, Sec. IV-B);
 *   LB_BC_OUTLET     x+ only: zero gradient, the node copies the populations
 *                    and moments of its neighbour (Sec. IV-B).
 * Both sides of an axis are periodic or both are bounded; inlet/outlet need a
 * periodic y axis; corners take the x-side wall's velocity and the
 * temperature of a Dirichlet x-side, else of a Dirichlet y-side, else the
 * adiabatic rule. */
typedef struct {
    int32_t kind; /* lb_bc_kind */
    int32_t pad_;
    double ux, uy, T;
    double amp, period;
} lb_side;

typedef struct {
    int32_t nx, ny;      /* node counts, boundary nodes included */
    int32_t storage;     /* lb_storage: population storage type */
    int32_t energy;      /* lb_energy: Eq. 18b/47 or internal energy (Eq. 38) */
    int32_t heating;     /* 1: viscous-heating coupling term of Eq. 47 (total energy only) */
    int32_t correction;  /* 1: correction term of Eq. 48-50 */
    int32_t coupled;     /* 1: theta-coupled Eq. 18; 0: decoupled theta = 1, p = rho R T0 (Eq. 8) */
    int32_t collision;   /* lb_collision */
    int32_t visc;        /* lb_visc */
    int32_t rho_extrap;  /* lb_rho_extrap: density of a wall node: LB_RHO_PRESSURE
                            extrapolates p = rho R T from the interior node with the
                            hydrostatic balance of the force, p_b = p_f
                            exp(g (y_f - y_b) / (R (T_f + T_b) / 2));
                            LB_RHO_DENSITY takes rho_f */
    double rho0, T0, R;  /* reference state; R * T0 = 1/3 */
    double b;            /* degrees of freedom, gamma = (b + 2) / b */
    double Pr;           /* Pr = (tau_f - 1/2) / tau_h; tau_hf = tau_f / (Pr - 1) */
    double tau_f;        /* shear relaxation time for LB_VISC_CONST_TAU, mu = (tau_f - 1/2) p */
    double s_e, s_zeta, s_q; /* rates of e, zeta, q in Eq. 40; s_e, s_zeta <= 0: tie to 1/tau_f */
    double tau_rho, tau_j;   /* relaxation times of the conserved moments (Eq. 40) */
    double mu_ref, T_ref;    /* viscosity mu(T_ref) of the other viscosity laws */
    double visc_n;           /* power law mu ~ T^n (Sec. IV-A) */
    double suth_S;           /* Sutherland constant S in lattice temperature units (Eq. 59) */
    double g;                /* gravity: force density a = (0, -rho g) (Sec. IV-C) */
    lb_side side[4];
} lb_params;

typedef struct lb_handle lb_handle;

/* Checks a parameter set.  LB_OK or LB_EINVAL (message in lb_last_error). */
lb_status lb_validate(const lb_params *p);

/* Bytes of device memory one grid needs: two population buffers of 18 planes
 * (row pitch nx rounded up to 64 nodes; inside each buffer the f^ half and
 * the h- half each keep the rows of their 9 populations next to each other,
 * [y][a][x]; lb_populations returns [18][ny][nx] whatever this internal
 * layout, and the lb_save image is opaque), a temperature snapshot plane and
 * reduction scratch.  0 when the parameters
 * are invalid. */
size_t lb_state_bytes(const lb_params *p);

/* Binds a grid to the caller's device buffer and HIP stream (a hipStream_t,
 * or NULL).  The device current on the calling thread is the one used.
 * The state is undefined until lb_init. */
lb_status lb_create(const lb_params *p, void *dev_state, size_t bytes, void *hip_stream, lb_handle **out);

/* Initial state: equilibrium populations of the given host fields
 * (rho, ux, uy, T as [ny][nx] doubles; a NULL field means rho0, 0, 0, T0).
 * Resets the time counter to 0 and forgets the temperature snapshot. */
lb_status lb_init(lb_handle *h, const double *rho, const double *ux, const double *uy, const double *T);

/* Advances n time steps (n >= 0), asynchronously on the stream.  Whole
 * batches of k steps (lb_set_graph_steps, default 32) replay a hipGraph of
 * k step launches captured on first use for the state's current buffer; the
 * rest are launched one by one.  Both give the same results bit for bit. */
lb_status lb_step(lb_handle *h, long n);

/* Launches per captured graph of lb_step: an even number up to 4096, or 0 to
 * launch every step from the host.  LB_EINVAL otherwise. */
lb_status lb_set_graph_steps(lb_handle *h, int k);

/* Current time step n. */
long lb_time(const lb_handle *h);

/* Macroscopic fields at the current time after the boundary treatment, into
 * host [ny][nx] doubles (NULL pointers are skipped).  Synchronises. */
lb_status lb_macros(lb_handle *h, double *rho, double *ux, double *uy, double *T);

/* Same fields as FP32 into device arrays with row pitch nx, asynchronously. */
lb_status lb_macros_device(lb_handle *h, float *rho, float *ux, float *uy, float *T);

/* Pre-collision populations at the current time after the boundary
 * treatment, into a host [18][ny][nx] double array.  Synchronises. */
lb_status lb_populations(lb_handle *h, double *out);

/* FP64 diagnostics at the current time: out[0] = sum of f^, out[1] = sum of
 * h-, out[2], out[3] = sum of e_x f^, e_y f^ (over all nodes and velocities),
 * out[4] = number of nodes with a non-finite moment, rho <= 0 or T <= 0,
 * out[5] = time step.  Returns LB_EUNSTABLE when out[4] > 0.  Synchronises. */
lb_status lb_diag(lb_handle *h, double out[6]);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, serving loops and harnesses that forbid hipMalloc): the
 * diagnostics of lb_diag written as 6 doubles to the caller's device array
 * dev_out (same meaning and values bit for bit), asynchronously on the
 * handle's stream, with no allocation, copy or synchronisation.  The partial
 * sums go to a static device array of the library (64 KiB, one per GPU,
 * kept until the process ends, shared by every call on that GPU): calls that
 * overlap on one GPU (other streams, other threads) race on it.  The caller
 * reads out[4] for unstable nodes.  LB_EINVAL on a null argument or a grid
 * whose reduction needs more than the array holds (never with the current
 * block count of at most 1024); LB_EHIP when a launch fails. */
lb_status lb_diag_noalloc(lb_handle *h, double *dev_out);

/* Convergence residual r = ||T - T_snap||_2 / ||T||_2 in FP64 against the
 * last snapshot (+inf when there is none); with update != 0 the current T
 * becomes the snapshot.  Synchronises. */
lb_status lb_residual(lb_handle *h, int update, double *r);

/* Checkpoint of the current state (populations, time, snapshot) into a host
 * buffer of lb_checkpoint_bytes() bytes, and back.  Both synchronise. */
size_t lb_checkpoint_bytes(const lb_handle *h);
lb_status lb_save(lb_handle *h, void *host_buf);
lb_status lb_load(lb_handle *h, const void *host_buf);

/* Launch tuning of the step kernel: rows per strip (power of two 1..256;
 * each block of wavefronts marches through one strip of rows), 0 restores
 * the automatic choice (8 rows with FP32 storage, 16 with FP16/BF16 and for
 * FP32 grids with walls, 2 in liblbddf_fp64.so, halved down to 1 while the
 * grid would give fewer than 4096 wavefronts, fully periodic grids, or 2048,
 * bounded ones).  Results do not depend on it.  Returns LB_EINVAL
 * for other values. */
lb_status lb_set_strip_rows(lb_handle *h, int rows);
int lb_strip_rows(const lb_handle *h);

/* Bandwidth reference (not part of the method): copies `bytes` from src to
 * dst, both device pointers, 16-byte aligned, not overlapping, bytes a
 * multiple of 16, with a STREAM-like kernel (16-byte vector loads, four in
 * flight per lane, non-temporal stores), asynchronously on hip_stream (NULL:
 * the null stream).  Timing it gives the practical memory ceiling beside the
 * nominal peak against which the step's algorithmic bytes per second are
 * read.  LB_EINVAL for null, misaligned or overlapping buffers; LB_EHIP when
 * the launch fails. */
lb_status lb_copy_probe(const void *src, void *dst, size_t bytes, void *hip_stream);

/* The HIP stream the handle launches on (a hipStream_t). */
void *lb_stream(const lb_handle *h);

/* Releases the handle (not the caller's device buffer).  NULL is ignored. */
void lb_destroy(lb_handle *h);

/* Message of the last failed call on this thread ("" if none). */
const char *lb_last_error(void);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of many grids of uneven sizes (cavities,
 * periodic boxes, grids with an outlet; not an inlet) in one packed launch
 * per time step.
 *
 * The caller hands the server one device pool; the server keeps the state of
 * every admitted request resident in it and admits queued requests first in,
 * first out as their byte footprint (lb_state_bytes), a slot (at most 512
 * resident grids) and room in the packed kernel's work list (2^18 items: one
 * per strip of each 64-column tile, or of each group of four tiles for FP32
 * grids at least 256 columns wide; strips of 4 rows, or of 2 for a batch that
 * would give fewer than 2048 wavefronts, and room is kept for 2) become free.  One lbs_advance call runs k steps of every
 * resident grid as hipGraphs of k launches of a packed kernel (the same
 * per-node step as lb_step): one for the grids in the cavity configuration
 * (internal energy, no heating term, coupled, correction, gravity, MRT, a
 * viscosity law other than constant tau), one for the others, so that a
 * grid's arithmetic depends on its own parameters only; then it reads every
 * grid's FP64 convergence
 * residual r = ||T - T_snap|| / ||T|| (snapshot k steps earlier; the first
 * at admission) in one copy,
 * retires grids that converged (r < tol), reached a plateau (r below 1e-2 of
 * its largest value and no new minimum for max(10, n/2) of its n checks so
 * far, minima counted from that maximum), reached max_steps (checked after
 * each batch, so a request runs to the next multiple of k) or became unstable,
 * stores their final fields on the host, frees their memory and admits
 * waiting requests.
 * Requests of one server share its storage type; inlet sides are not served
 * (the packed step is compiled for grids with walls, outlet or periodic
 * sides).
 * One server must not be used by two threads at once.
 * ------------------------------------------------------------------------ */
typedef struct lbs_server lbs_server;

typedef enum {
    LBS_QUEUED = 0,
    LBS_RUNNING = 1,
    LBS_CONVERGED = 2,
    LBS_PLATEAU = 3,
    LBS_STEP_CAP = 4,
    LBS_UNSTABLE = 5
} lbs_state;

/* Bytes of the pool the server keeps for its slot and work tables. */
size_t lbs_pool_overhead(void);

/* Server over a caller-owned, 256-byte aligned device pool of pool_bytes
 * bytes; storage is an lb_storage, k_steps the steps per batch. */
lb_status lbs_create(void *dev_pool, size_t pool_bytes, int storage, int k_steps, void *hip_stream, lbs_server **out);

/* Queues a request (host fields as in lb_init, NULL: rest state); *id
 * receives its handle.  LB_ENOMEM when it cannot fit the pool at all,
 * LB_EINVAL when its work items alone exceed the work list. */
lb_status lbs_submit(lbs_server *s, const lb_params *p, const double *rho, const double *ux, const double *uy,
                     const double *T, double tol, long max_steps, long *id);

/* Admission, one packed batch of k steps over all resident grids, residual
 * checks, retirement and admission again.  Synchronises the stream.  Reports
 * the resident and queued counts at the start of the batch. */
lb_status lbs_advance(lbs_server *s, int *n_resident, int *n_queued);

/* State (lbs_state), steps done, last residual and the submit, admit and
 * finish times (seconds since lbs_create; -1 until reached) of a request. */
lb_status lbs_poll(lbs_server *s, long id, int *state, long *steps, double *residual, double times[3]);

/* Final fields of a finished request (LB_EBUSY while queued or running). */
lb_status lbs_result(lbs_server *s, long id, double *rho, double *ux, double *uy, double *T);

/* Forgets a finished request and its stored fields. */
lb_status lbs_release(lbs_server *s, long id);

/* out = {batches, node updates, seconds inside lbs_advance batches, finished
 * requests, free pool bytes, queued requests}. */
lb_status lbs_stats(lbs_server *s, double out[6]);

/* Releases the server (not the caller's pool). */
void lbs_destroy(lbs_server *s);

#ifdef __cplusplus
}
#endif
#endif /* LBDDF_H */
