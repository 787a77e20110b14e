/*
 * sl.h -- C ABI of the MI355X semi-Lagrangian spectral transport library.
 *
 * The library advances u_t + a . grad u = 0 (advective form) or
 * phi_t + div(a phi) = 0 (conservative form, paper section 2, eq. 2.3/2.4)
 * on a uniform mesh of K quadrilateral (2D) or interval (1D) elements of
 * order N (n = N + 1 nodes per direction) with the explicit semi-Lagrangian
 * DSEM step of Natarajan & Jacobs (arXiv 1910.06476, section 4): particles
 * seeded at the Gauss nodes (section 4.1), moved by one explicit Runge-Kutta
 * step (section 4.2, eq. 4.4a / 4.8), remapped to the fixed nodes (section
 * 4.3, eq. 4.9; 2D: eq. 5.4), and corrected by a least-squares fit
 * constrained by the upwind interface values (eq. 4.12a) and optionally by
 * local mass (eq. remap_mass) and energy (eq. remap_energy) targets
 * (eq. matrix_a).
 *
 * Conventions
 *   - Every entry point returns sl_status (0 = SL_OK); no C++ exception
 *     crosses the ABI.
 *   - Pointers documented "host" are ordinary host memory owned by the
 *     caller; the library copies what it needs and keeps no reference.
 *   - Field layout (u0, sl_read output, velocity components, divergence):
 *     element-major, double, element index k = ix + kx * iy, node index
 *     p = i + n * j with i along x (1D: p = i).  Element (ix, iy) covers
 *     [x0 + ix dx, x0 + (ix+1) dx] x [y0 + iy dy, y0 + (iy+1) dy].
 *   - Node positions inside an element are given by sl_node_coords.
 *   - A mesh is used by one host thread at a time; distinct meshes are
 *     independent.  All device work of a mesh runs on its stream.
 */
#ifndef SL_H
#define SL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sl_status;

enum {
    SL_OK = 0,
    SL_E_INVALID = 1,   /* bad argument or descriptor; nothing changed          */
    SL_E_NOMEM = 2,     /* device allocation failed; nothing left allocated      */
    SL_E_DEVICE = 3,    /* a HIP runtime call failed                             */
    SL_E_STATE = 4,     /* call not valid in the mesh's current state            */
    SL_E_CFL = 5,       /* time step lets a particle leave its element           */
    SL_E_NONFINITE = 6, /* NaN/Inf in inputs or produced by a step               */
    SL_E_SINGULAR = 7,  /* a remap or constraint system had a zero pivot          */
    SL_E_NOCONV = 8     /* energy Picard iteration hit its cap above tolerance   */
};

enum { SL_NODES_GL = 0, SL_NODES_CG = 1 };          /* Gauss-Legendre / Chebyshev-Gauss */
/* Boundary conditions.  Periodicity pairs opposite sides, so in 2D it is
 * chosen per direction: SL_BC_PERIODIC_X wraps the left and right sides
 * onto each other and takes ghost values on the bottom and top sides;
 * SL_BC_PERIODIC_Y the other way round. */
enum { SL_BC_PERIODIC = 0, SL_BC_GHOST = 1, SL_BC_PERIODIC_X = 2, SL_BC_PERIODIC_Y = 3 };
enum { SL_FORM_ADVECTIVE = 0, SL_FORM_CONSERVATIVE = 1 };
enum { SL_PREC_FP64 = 0, SL_PREC_FP32_REFINED = 1, SL_PREC_BF16_REFINED = 2 };
enum { SL_C_BOUNDARY = 1, SL_C_MASS = 2, SL_C_ENERGY = 4 };
enum { SL_MODE_HARD = 0, SL_MODE_SOFT = 1 };
enum { SL_IFACE_INTERP = 0, SL_IFACE_BACKTRACK = 1 };

/* Mesh descriptor (sl_create_mesh).
 *   dim        1 or 2
 *   kx, ky     elements per direction (ky = 1 in 1D); kx * ky <= 2^26
 *   order      polynomial order N >= 1 (n = N + 1 nodes per direction);
 *              1D: N <= 16, 2D: N <= 16 (2D N = 16: FP64 and boundary
 *              rows only)
 *   nodes      SL_NODES_GL (default) or SL_NODES_CG (paper, eq. gaussquad)
 *   bc         SL_BC_PERIODIC, or SL_BC_GHOST (inflow values from sl_set_ghost
 *              on every side), or in 2D SL_BC_PERIODIC_X / SL_BC_PERIODIC_Y
 *              (periodic in one direction, ghost values on the two sides
 *              of the other)
 *   form       SL_FORM_ADVECTIVE or SL_FORM_CONSERVATIVE
 *   precision  SL_PREC_FP64, SL_PREC_FP32_REFINED or SL_PREC_BF16_REFINED
 *              (2D only: the preconditioner of the remap solve is stored
 *              and applied in FP32, or with BF16 entries and operands and
 *              FP32 accumulation, while residuals and iterates stay FP64, so
 *              the solve still converges to the FP64 solution, in more
 *              sweeps; 1D and 2D order 16 reject both)
 *   x0,x1,y0,y1 box (y ignored in 1D), x1 > x0, y1 > y0
 *   u0         host, K * n^dim initial values (layout above)
 *   stream     hipStream_t to run on, or NULL for a stream the mesh creates
 *   orders     NULL, or (2D, periodic) host array of K per-element orders
 *              N_e in 1..16 for a mixed-order mesh: element e then has
 *              n_e = N_e + 1 nodes per direction, `order` is ignored, and
 *              every per-node array (u0, velocity components, the field of
 *              sl_read) holds the elements one after another, n_e^2 values
 *              each, node i + n_e j.  Elements of different orders are
 *              coupled through the face values: the upwind side's edge
 *              polynomial is evaluated at the element's own edge nodes.
 *              Mixed-order meshes take boundary rows only (HARD or SOFT);
 *              their steps run as a captured HIP graph. */
typedef struct {
    int32_t dim, kx, ky, order;
    int32_t nodes, bc, form, precision;
    double x0, x1, y0, y1;
    const double* u0;
    void* stream;
    const int32_t* orders;
} sl_mesh_desc;

/* Step options (sl_step); a NULL pointer means all defaults.
 *   rk            explicit Runge-Kutta order 1..4 (Euler, Heun, Kutta-3,
 *                 classical RK4); default 4
 *   constraints   mask of SL_C_*; default SL_C_BOUNDARY
 *   mode          SL_MODE_HARD (KKT: rows hold exactly, default) or
 *                 SL_MODE_SOFT (the paper's stacked least squares)
 *   energy_maxit  Picard iterations cap for the energy row (default 50)
 *   refine_steps  reserved (the remap refinement runs to its own stop test);
 *                 must be >= 0
 *   iface         interface values at t^{n+1} (section 4.3): SL_IFACE_INTERP
 *                 (default), the remapped polynomial at the element edge (eq.
 *                 remap_bnd); or SL_IFACE_BACKTRACK, phi^n at the foot of the
 *                 characteristic traced back over dt from the edge point with
 *                 the particles' RK tableau (eq. 4.11; times the source
 *                 factor in the conservative form).  Either is computed on
 *                 the side of each face where the flow leaves (both sides
 *                 where the face speed vanishes) and selected by upwinding
 *                 (eq. 4.12a).  Mixed-order meshes take SL_IFACE_INTERP only.
 *   energy_tol    Picard stop |phi^(k) - phi^(k-1)|_max < tol (default 1e-8, the
 *                 paper's; 0 = always run energy_maxit iterations) */
typedef struct {
    int32_t rk, constraints, mode, energy_maxit, refine_steps, iface;
    double energy_tol;
} sl_step_opts;

/* Statistics returned by sl_read (accumulated since the last sl_read).
 *   resid_*   largest |row . phi - target| seen (boundary: in the 2D
 *             least-squares sense, the corner dependencies make it nonzero)
 *   max_picard largest number of energy-row solves in one element and step
 *   flags     bit0 non-finite, bit1 particle left element, bit2 singular
 *             system, bit3 Picard not converged
 *   vel_terms number of Chebyshev terms (per direction in 2D) of the
 *             velocity series the kernels evaluate: trailing terms below
 *             2^-46 of max(the element series' absolute sum, mesh max |a|)
 *             -- the rounding noise of the nodal-to-modal transform -- are
 *             skipped
 *   refine_resid      2D: largest estimated error left by the iterative
 *                     remap solve (eq. 5.4): its last correction times the
 *                     observed contraction, relative to max |phi*| of the
 *                     element; 0 in 1D
 *   remap_sweeps_max  2D: most defect-correction sweeps one element needed
 *   remap_sweeps_mean 2D: sweeps per element and step, averaged */
typedef struct {
    double t;
    int64_t steps;
    double mass, energy;
    double resid_boundary, resid_mass, resid_energy;
    double refine_resid;
    int32_t max_picard;
    int32_t flags;
    int32_t vel_terms;
    int32_t remap_sweeps_max;
    double remap_sweeps_mean;
} sl_stats;

typedef struct sl_mesh sl_mesh;

/* Create a mesh: validates the descriptor, builds the reference-element
 * tables, allocates device state and copies u0 (host) to the device.
 * On error *out is NULL and nothing stays allocated.
 * Errors: SL_E_INVALID, SL_E_NOMEM, SL_E_DEVICE, SL_E_NONFINITE (u0). */
sl_status sl_create_mesh(const sl_mesh_desc* desc, sl_mesh** out);

/* Set the (steady) velocity field.  a: host, dim * K * n^dim values,
 * component-major (all x components, then all y components), given at the
 * Gauss nodes as a DSEM solver supplies it (section 4.2); the velocity off
 * the nodes is the element's Lagrange interpolant.  div_a: host, K * n^dim
 * nodal values of div(a), or NULL to take the divergence of the interpolant.
 * Copies both; derived tables (modal coefficients, face velocities) are
 * built on the device.  Errors: SL_E_INVALID, SL_E_NONFINITE, SL_E_DEVICE. */
sl_status sl_set_velocity(sl_mesh* m, const double* a, const double* div_a);

/* Ghost (outside) values at the domain boundary for meshes with ghost
 * sides (SL_BC_GHOST, SL_BC_PERIODIC_X, SL_BC_PERIODIC_Y).
 * g: host, nrows rows of nghost values; row r holds the outside state at
 * time t + r dt where t is the mesh time at this call, so the i-th following
 * step reads rows i and i+1 (clamped to the last row; nrows = 1 is a steady
 * ghost).  Row layout -- 1D: [left, right]; 2D: left edge (ky * n values,
 * by iy then node j), right edge (ky * n), bottom edge (kx * n, by ix then
 * node i), top edge (kx * n); the values of periodic sides are neither
 * read nor checked.
 * Errors: SL_E_STATE (periodic mesh),
 * SL_E_INVALID, SL_E_NOMEM. */
sl_status sl_set_ghost(sl_mesh* m, const double* g, int32_t nrows);

/* Number of ghost values per row (see sl_set_ghost). */
int32_t sl_ghost_count(const sl_mesh* m);

/* Advance nsteps explicit SL steps of length dt, asynchronously on the
 * mesh's stream.  Validated before any launch (state unchanged on error):
 * SL_E_STATE (no velocity, or ghost mesh without ghost values),
 * SL_E_INVALID (dt <= 0, nsteps < 0, bad options; 1D: more rows than n;
 * 2D HARD with boundary rows: more mass/energy rows than (n-2)^2, the
 * dimension of the null space of the 4n boundary rows of rank 4n-4; 2D
 * order 16: mass or energy rows),
 * SL_E_CFL (max |a_d| dt > gap_d dx_d for some direction d, gap =
 * distance from the element edge to the first node: the paper's time-step
 * restriction, eq. 1d_delt_condition and eq. 2d_delt_condition, which admits
 * equality). */
sl_status sl_step(sl_mesh* m, double dt, int32_t nsteps, const sl_step_opts* opts);

/* Synchronise the mesh's stream and copy the field to u_out (host, K * n^dim
 * doubles, same layout as u0; may be NULL).  st (may be NULL) receives the
 * statistics accumulated since the previous sl_read, which are then reset.
 * Returns SL_E_NONFINITE / SL_E_SINGULAR / SL_E_NOCONV when the matching
 * flag was raised (the copy has still been made), else SL_OK or
 * SL_E_DEVICE. */
sl_status sl_read(sl_mesh* m, double* u_out, sl_stats* st);

/* Free the mesh's device memory and stream (if it created one). */
sl_status sl_destroy_mesh(sl_mesh* m);

/* Human-readable name of a status code (static string). */
const char* sl_status_string(sl_status s);

/* Largest dt allowed by the time-step restriction, times cfl (0 < cfl <= 1);
 * 0 if no velocity is set, or the mesh is NULL. */
double sl_max_dt(const sl_mesh* m, double cfl);

/* Reference node positions xi[n] on [0,1] and quadrature weights w[n]
 * (summing to 1) of a node family; both host arrays of n doubles.
 * Errors: SL_E_INVALID (unknown family, n < 1 or n > 32). */
sl_status sl_node_coords(int32_t nodes, int32_t n, double* xi, double* w);

/* Device pointer of the mesh's field (K * n^dim doubles, layout above) and
 * the mesh's stream, for callers that keep data on the device.  The pointer
 * stays valid until sl_destroy_mesh; writes through it must be ordered on
 * the mesh's stream. */
sl_status sl_device_field(sl_mesh* m, double** d_phi, void** stream);

/* Per-kernel timing with HIP events on the mesh's stream.  When enabled,
 * every kernel launch of sl_step is bracketed by events (a mixed-order mesh
 * then steps without its captured graph); sl_kernel_time synchronises and
 * returns the summed milliseconds and the launch count of kernel 'which'
 * since the last reset: 0 = 1D advect, 1 = 1D constrain, 2 = 2D advect+solve
 * (a mixed-order mesh: its whole step), 3 = 2D constrain, 4 + b = the
 * advect+solve of bucket b of a mixed-order mesh, 20 + b = its constrain
 * (buckets in ascending order, b < 16), 36 = the 2D targets of mass and
 * energy rows, 37 = the 2D face backtraces of SL_IFACE_BACKTRACK (uniform
 * 2D meshes).  Errors: SL_E_INVALID. */
sl_status sl_set_profiling(sl_mesh* m, int32_t enable);
sl_status sl_kernel_time(sl_mesh* m, int32_t which, double* total_ms, int64_t* launches);

/* Per order bucket of a mixed-order mesh (bucket 0 of a uniform mesh is the
 * whole mesh): its nodes per direction n, element count, velocity series
 * terms per direction the kernels evaluate, and its mean remap (eq. 5.4)
 * sweeps per element and step since the last sl_read (call it before
 * sl_read, which resets the statistics; 0 in 1D).  Synchronises the mesh's
 * stream.  Any output pointer may be NULL.  Errors: SL_E_INVALID,
 * SL_E_DEVICE. */
sl_status sl_bucket_stats(sl_mesh* m, int32_t bucket, int32_t* n, int32_t* count, int32_t* vel_terms,
                          double* sweeps_mean);

/* Device bytes a mesh with descriptor d holds (all its buffers, and
 * ghost_rows rows of ghost values for a GHOST mesh), for admission by
 * memory budget.  d->u0 is not read.  Errors: SL_E_INVALID. */
sl_status sl_mesh_bytes(const sl_mesh_desc* d, int32_t ghost_rows, size_t* bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): nsteps 1D
 * steps, the work sl_step does on a 1D mesh, on the caller's device
 * buffers, with no mesh and no allocation.  Each call prepares the velocity
 * (its Chebyshev series, divergence and face speeds), then runs the steps on
 * `stream` (hipStream_t, or NULL for the null stream) and returns without
 * synchronising.  The kernels' scratch memory is one fixed device array of
 * the library (about 54 MB, held on each GPU the library runs on until the
 * process ends); its device address is looked up, and the reference tables
 * of every order are copied into it, at the first call on a device (a
 * synchronous copy).  Every call on one GPU shares that array and it keeps
 * the last call's contents, so calls that overlap on one GPU (other streams
 * or host threads) race and must be ordered by the caller.
 *   K, order   elements and order N: 1 <= K <= 65536, 1 <= N <= 16,
 *              K (N + 1) <= 1114112; larger sizes are rejected with
 *              SL_E_INVALID before any device call
 *   nodes, bc, form   as in sl_mesh_desc (bc: SL_BC_PERIODIC or SL_BC_GHOST)
 *   x0, x1     the interval
 *   phi_in     device, K (N + 1) values, the field at t (layout of u0)
 *   phi_out    device, K (N + 1) values, the field after nsteps steps; may
 *              equal phi_in
 *   a          device, K (N + 1) nodal velocity values
 *   div_a      device, K (N + 1) nodal values of div(a), or NULL to take the
 *              divergence of the interpolant
 *   amax       host value: the largest |a| over the nodes (the stagnation
 *              threshold 1e-12 amax and the time-step check, as sl_step)
 *   ghost      device, SL_BC_GHOST only: nsteps + 1 rows of [left, right]
 *              outside values, row r at time t + r dt
 *   dt, nsteps, opts   as sl_step (opts NULL: defaults); nsteps = 0 copies
 *              phi_in to phi_out
 *   stats      device, 4 doubles or NULL: the largest boundary, mass and
 *              energy residuals and energy sweep count over the call's steps
 *   flags      device, 1 int32 or NULL: the call's flag bits (sl_stats.flags)
 * Results equal those of sl_create_mesh + sl_set_velocity + sl_step on the
 * same data to rounding (this call evaluates the whole velocity series,
 * sl_step only its effective degree).  Errors: SL_E_INVALID, SL_E_CFL,
 * SL_E_DEVICE. */
sl_status sl_step1d_static(int32_t K, int32_t order, int32_t nodes, int32_t bc, int32_t form, double x0, double x1,
                           const double* phi_in, double* phi_out, const double* a, const double* div_a, double amax,
                           const double* ghost, double dt, int32_t nsteps, const sl_step_opts* opts, double* stats,
                           int32_t* flags, void* stream);

/* ------------------------------------------------------------------------
 * Request loop (continuous batching of independent problems on one GPU).
 *
 * A request is a whole transport problem: mesh descriptor (with u0),
 * velocity, optional divergence and ghost rows, dt, step count and options;
 * all host arrays are copied at submission.  Requests wait in arrival order
 * and are admitted while fewer than max_active run and the device memory
 * they need (sl_mesh_bytes) fits within hbm_budget.  An admitted request
 * gets its own mesh, carved from one block of a device arena that the
 * server allocates once, at its first admission (hbm_budget plus 8.25 KiB
 * per slot, at most 90% of the device memory then free), and one of the
 * server's streams (one per slot).  Small requests (whose advect launch
 * has fewer than 2048 workgroups, so that alone they leave the device
 * partly idle) whose steps share a kernel variant (same dimension and
 * order; boundary rows; interpolated face values; 2D order 3 and up; the
 * same advect variant) are stepped together: each step of the group is
 * one launch of each step kernel over the elements of all its members
 * with steps left, on the group's stream, and members join and leave
 * between such steps.  Other requests queue all their steps at once on
 * their own stream.  The work of the admitted
 * requests overlaps on the device.  Results do not depend on what else
 * runs: every kernel is deterministic, and a block of a batched launch
 * works for one request on its own buffers, so a field is the same, bit
 * for bit, alone and in any mix.
 *
 * The loop (admission, set-up, stepping, retirement) runs on host threads
 * of the server's own (one for set-up and retirement, with up to three
 * helpers while it sets up several requests at once; one feeding the
 * device), started by the first sl_server_progress or sl_server_drain;
 * the caller only submits and collects.  Calls on one
 * server may come from several host threads, except sl_server_destroy,
 * which no other call on that server may overlap.
 * ------------------------------------------------------------------------ */
typedef struct sl_server sl_server;

enum { SL_SERVER_NO_BATCH = 1 };

typedef struct {
    int32_t max_active;   /* requests on the device at once, 1..64 */
    int32_t flags;        /* 0, or SL_SERVER_NO_BATCH: every request on its own stream */
    size_t hbm_budget;    /* bytes of device memory admitted requests may hold */
} sl_server_desc;

typedef struct {
    sl_mesh_desc mesh;    /* mesh.u0: host initial field; mesh.stream ignored;
                             mesh.orders must be NULL (uniform meshes only) */
    const double* a;      /* host nodal velocity, layout of sl_set_velocity */
    const double* div_a;  /* host nodal divergence or NULL */
    const double* ghost;  /* host ghost rows (GHOST meshes), layout of sl_set_ghost */
    int32_t ghost_rows;
    int32_t nsteps;       /* steps of length dt */
    double dt;
    sl_step_opts opts;
} sl_request;

typedef struct {
    double queue_us;      /* host time from submission to admission */
    double total_us;      /* host time from submission to retirement */
    double device_ms;     /* device time from before the first to after the last step */
    size_t bytes;         /* device memory the request held */
    int64_t admit_seq;    /* order of admission among the server's requests (0 first), -1 if never admitted */
} sl_request_timing;

/* Errors: SL_E_INVALID (max_active outside 1..64, zero budget, unknown
 * flags), SL_E_NOMEM, SL_E_DEVICE. */
sl_status sl_server_create(const sl_server_desc* d, sl_server** out);

/* Queue a request; *id names it in sl_server_result.  Errors: SL_E_INVALID
 * (bad request or descriptor, or a mixed-order descriptor: mesh.orders is
 * not NULL), SL_E_NOMEM (it could never fit the budget, or host memory). */
sl_status sl_server_submit(sl_server* s, const sl_request* r, int64_t* id);

/* Non-blocking: starts the loop at the first call, then reports.  The loop
 * retires finished requests (field and statistics copied to host memory,
 * mesh freed) and admits waiting ones in arrival order; a request whose
 * set-up or step validation fails is finished with that status.  *active
 * (requests holding a slot: in set-up, stepping, or being retired) and
 * *waiting (may be NULL) receive the counts.  Errors: SL_E_INVALID, and
 * the loop's first device error (SL_E_DEVICE), which stops it; SL_E_NOMEM
 * if its threads cannot start. */
sl_status sl_server_progress(sl_server* s, int32_t* active, int32_t* waiting);

/* Start the loop if needed and block until nothing is active or waiting.
 * Errors: those of sl_server_progress. */
sl_status sl_server_drain(sl_server* s);

/* Result of a finished request: the field (host, K * n^dim doubles; may be
 * NULL), its statistics and timing (may be NULL); then the request is
 * forgotten.  Returns the request's own status (that of its sl_read or of
 * its failed set-up), SL_E_STATE if it is not finished, SL_E_INVALID for an
 * unknown id. */
sl_status sl_server_result(sl_server* s, int64_t id, double* u_out, sl_stats* st, sl_request_timing* tm);

/* Per-step device latency over all retired requests' steps (the time
 * between the events that bracket consecutive steps of one request, so it
 * includes waiting behind the other requests' work; for batched requests,
 * the time of the group step that carried it): p50 and p99 in ms; the
 * number of samples and the DOF-updates of the retired requests.  Errors:
 * SL_E_INVALID. */
sl_status sl_server_latency(sl_server* s, double p50_p99[2], int64_t* samples, int64_t* dof_updates);

/* Batched steps so far: the number of group steps launched (one launch of
 * each step kernel each) and the request steps they carried.  Errors:
 * SL_E_INVALID. */
sl_status sl_server_batching(sl_server* s, int64_t* launches, int64_t* member_steps);

/* Stop the loop (a set-up in progress is completed first), wait for the
 * device work already queued, free everything.  Errors: SL_E_INVALID. */
sl_status sl_server_destroy(sl_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SL_H */
